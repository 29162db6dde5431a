// Shared declarations of the gfx950 phaseless-AFQMC library: complex helpers,
// error plumbing, the system/walker objects and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>
#include "afq.h"

// ---------------------------------------------------------------------------
// error handling: internal functions return afq_status; the C ABI stores the
// message in a thread-local string.
// ---------------------------------------------------------------------------
void afq_set_error(const std::string& msg);

#define AFQ_TRY_HIP(expr)                                                        \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      afq_set_error(std::string(#expr) + ": " + hipGetErrorString(e_));          \
      return e_ == hipErrorOutOfMemory ? AFQ_E_NOMEM : AFQ_E_HIP;                \
    }                                                                            \
  } while (0)

inline int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return AFQ_OK;
  afq_set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? AFQ_E_NOMEM : AFQ_E_HIP;
}

#define AFQ_CHECK(cond, code, msg)                                               \
  do {                                                                           \
    if (!(cond)) {                                                               \
      afq_set_error(msg);                                                        \
      return (code);                                                             \
    }                                                                            \
  } while (0)

#define AFQ_RET(expr)                                                            \
  do {                                                                           \
    int r_ = (expr);                                                             \
    if (r_ != AFQ_OK) return r_;                                                 \
  } while (0)

// ---------------------------------------------------------------------------
// complex arithmetic on HIP vector types (double2 / float2 = re, im)
// ---------------------------------------------------------------------------
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using cplx_t = typename cvec<T>::type;

__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm keeps the intermediate quotient in range
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.y + b.x * r;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}
__device__ inline double2 clog(double2 a) { return make_double2(0.5 * log(cabs2(a)), atan2(a.y, a.x)); }

// ---------------------------------------------------------------------------
// device buffer owned by the library
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int alloc(size_t n);
  void free();
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
  ~DevBuf() { free(); }
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  void swap(DevBuf& o) noexcept {   // exchange the allocations (no device work)
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
  }
};

// ---------------------------------------------------------------------------
// packed operand layout of the exchange GEMM  C[(n,a)][(w,part,b)] = sum_k A B
//   A rows (n, a): n * np + a, a < N (rows a >= N are zero), k < kp; stored
//   row-major, or chunk-major (all rows of k-chunk 0, then of chunk 1, ...)
//   B rows (w, part, b): per walker 2*np rows, part 0 = Re, 1 = Im
//   real trial: k runs over M orbitals;  complex trial: k over 2M
//   (A = [Lt_re | Lt_im], B = [[Th_re, Th_im], [-Th_im, Th_re]])
// ---------------------------------------------------------------------------
struct PackShape {
  int n = 0;      // electrons of this spin
  int np = 0;     // rows per block: n rounded up to 16, or n (stacked layout)
  int ke = 0;     // contraction length (M or 2M)
  int kp = 0;     // ke rounded up to the k-chunk
  bool big = false;  // stacked layout of the one-wave-per-SIMD kernel
  int pad = 0;    // zero rows after the last block (A and B)
  int kcm = 0;    // 0: row-major (row * kp + k); else chunk-major ((k / kcm) * rows + row) * kcm + k % kcm
  long rows_b(int nw) const { return (long)nw * 2 * np + pad; }
};

int exch_kchunk(int prec);

struct afq_system_s {
  int M = 0, n_up = 0, n_dn = 0, X = 0, ntot = 0;
  double e_core = 0.0;
  int prec = AFQ_FP64;
  hipStream_t stream = nullptr;
  int device = 0;
  bool real_trial = true;
  DevBuf h1, chol, phi;        // f64 inputs (phi complex M x ntot)
  DevBuf chol32t;              // reduced modes: upper block triangle of L as FP32 packed rows e of [n / 16][e][n % 16]
  DevBuf tri8;                 // its 8 x 8 block pairs (bm << 16 | bk, bm <= bk), 64 rows e each (FP32 ring)
  DevBuf chol3;                // split-BF16x3 mode: the same rows e as BF16 hi / lo planes [n / 32][e][n % 32]
  DevBuf b1x;                  // reduced modes: (B1 - I) FP32 packed rows m, for W + (B1 - I) W
  double b1x_dt = -1.0;
  DevBuf b1x3;                 // split-BF16x3 mode: the same as BF16 hi / lo planes
  double b1x3_dt = -1.0;
  int b1x3_tile = -1;          // the product tile its rows were padded for
  int b3_tile = -1;            // split-BF16x3 Taylor and B1 product tile (index into the tile table; -1: the
                               // padded-work model chooses; afq_autotune or afq_system_set_propagator_tile pin it)
  DevBuf lt32[2];              // split-BF16x3, real trial: Lt rows n of each spin, FP32 packed [J / 16][n][J % 16]
  bool lt_share = false;       // the two trial blocks are equal: lt32[1] is not built, the force bias contracts
                               // Theta_up + Theta_dn with lt32[0]
  DevBuf hp;                   // h' = h - 1/2 sum L L   (M x M f64)
  DevBuf B1;                   // exp(-dt h'/2)          (M x M f64), or exp(-dt h_mf/2) with a background
  double B1_dt = -1.0;
  bool mf_on = false;          // mean-field background subtraction
  DevBuf vmf;                  // X f64: the background vector c_n
  DevBuf hp_mf;                // h' + sum_n c_n L^n (M x M f64)
  unsigned b1_serial = 0;      // bumped when the one-body factor changes other than through dt
  DevBuf ht;                   // (T^H h)  ntot x M complex
  DevBuf Lt;                   // (T^H L^n) X x ntot x M complex
  DevBuf LtRe;                 // real part of Lt (real trial, split-BF16x3 force bias)
  DevBuf phir;                 // real trial: Re T (M x ntot f64), the overlap kernel's trial operand
  DevBuf apack[2];             // packed A operand per spin (precision of prec)
  DevBuf apack_lo[2];          // BF16x3 low parts
  int apack_prec = -1;
  PackShape ps[2];
  // orthogonal multi-determinant trial (msd_n == 0: the single determinant phi)
  int msd_n = 0;               // determinants
  int msd_no[2] = {0, 0};      // active holes per spin
  int msd_nexc[2] = {0, 0};    // distinct excitations per spin
  int msd_nv = 0;              // active virtual orbitals (both spins)
  int msd_nr = 0;              // rows per operator: max(n_up, n_dn) reference + msd_nv virtual
  size_t msd_lds = 0;          // dynamic LDS bytes of the determinant-sum kernel
  DevBuf msd_cconj;            // n_det complex: conj(c_I)
  DevBuf msd_pair;             // n_det x 2 int: excitation index of each spin
  DevBuf msd_exc[2];           // n_exc x MSD_EXC int: rank, hole slots, particle slots, hole columns
  DevBuf msd_hact[2];          // n_o int: reference column of every active hole
  DevBuf msd_csr_off[2];       // n_exc + 1 int: determinants of each excitation (offsets)
  DevBuf msd_csr_det[2];       // n_det int: determinant indices grouped by excitation
  DevBuf msd_cvh;              // msd_nv x M complex: C_V^H (active virtual orbitals)
  DevBuf msd_lact;             // (X + 1) x msd_nr x M complex: [C_ref^H; C_V^H] L^g, g = X is h1
  // k-point-blocked Cholesky (kp_nk > 0): orbital (k, i) -> k m + i; trial
  // columns (k, a) k-major per spin; 2 nk xq fields (x for the Hermitian parts
  // a = (L + L^+)/2, y for b = (L - L^+)/(2i) of every vector (Q, n))
  int kp_nk = 0, kp_m = 0, kp_xq = 0, kp_nu = 0, kp_nd = 0;   // per k-point electrons
  size_t kp_lds = 0;           // dynamic LDS bytes of the k-point trace kernel
  DevBuf kp_kq;                // nk x nk int: kq[Q][k] = k + Q
  DevBuf kp_kd;                // nk x nk int: kd[a][b] = the Q with b + Q = a
  DevBuf kp_L;                 // [Q][n][k][i][l] complex: L^{Q,k}_n, block (k + Q, k)
  DevBuf kp_Lt;                // [Q][k][n][a][l] complex: (T^{k+Q})^H L^{Q,k}_n (both spins' a)
  DevBuf kp_Ltd;               // [Q][k][n][a][l] complex: (T^k)^H (L^{Q,k}_n)^+
  DevBuf kp_h;                 // M x M complex h (block diagonal)
  DevBuf B1c;                  // M x M complex B1 = exp(-dt h'/2) (block diagonal)
  std::vector<double2> kp_hp;  // h' blocks on the host, nk x m x m
  // four-index exchange (split-BF16x3, real trial): W'' planes per distinct spin block
  int eri_form = AFQ_EXCH_AUTO;
  bool eri_ready = false;      // planes built for the current configuration
  bool eri_share = false;      // both spins use block 0 (equal trial blocks)
  bool eri_declined = false;   // the automatic choice said no for this configuration
  int eri_prec = -1;           // precision the tensor was built for (AFQ_BF16X3 or AFQ_FP64)
  DevBuf eri_w[2];             // BF16x3: hi and lo planes, chunk-major [chunk][rows][32] bf16;
                               // FP64: the full symmetric W' (N M x N M f64)
  DevBuf eri_units[2];         // work units (row block, first chunk, chunks, interval)
  int eri_nunit[2] = {0, 0};
  std::vector<int> eri_units_host[2];   // the same, on the host (the walkers' launch layouts)
  unsigned eri_gen = 0;        // changes whenever the units are rebuilt
  unsigned version = 0;        // bumped when the step's kernel sequence changes (batches capture again)
  int nspin_n(int s) const { return s == 0 ? n_up : n_dn; }
  int spin_off(int s) const { return s == 0 ? 0 : n_up; }
};

struct afq_walkers_s {
  afq_system sys = nullptr;
  int nw = 0;
  uint64_t counter = 0;
  DevBuf W, Wn;                // walkers and the propagated copy (nw x M x ntot c128)
  DevBuf weights;              // nw f64
  DevBuf alive;                // nw int32
  DevBuf killed;               // 1 x int64: walkers killed so far
  DevBuf d_counter;            // 1 x uint64: step counter on the device (keys the Philox fields)
  int exch_var[2] = {-1, -1};  // exchange launch variant per spin chosen by the autotuner (-1: cached/default)
  double fb_cap = 0.0;         // force-bias modulus cap (0: off)
  double w_cap = 0.0;          // weight cap (0: off)
  DevBuf comb_cum, comb_src;   // population control scratch: running weight sums, source indices
  DevBuf comb_out;             // 2 doubles: total weight, new common weight
  // back-propagation window (bp_n < 0: none)
  int bp_n = -1;               // window length in steps
  int bp_rec = 0;              // steps recorded so far
  uint64_t bp_start = 0;       // step counter when the window opened
  double bp_dt = -1.0;         // time step of the recorded steps
  int bp_order = 0;            // Taylor order of the recorded steps
  int bp_prec = -1;            // precision of the recorded coefficients
  unsigned bp_b1 = 0;          // system b1_serial when the window opened
  DevBuf bp_W0;                // walkers when the window opened (nw x M x ntot c128)
  DevBuf bp_coef, bp_tmp;      // bp_n x nw x X conj(c) (f64 or f32 complex); gather scratch
  DevBuf bp_psi;               // back-propagated trial (nw x M x ntot c128)
  DevBuf bp_stats;             // 2 doubles: sum of weights, singular count
  // per-step scratch
  DevBuf S, Sinv;              // per (w, spin): n x n complex (max n^2 stride)
  DevBuf Sinv_new;             // S^-1 of the propagated walkers (carried to the next step)
  bool s_carried = false;      // Sinv and logdet are those of the current W (set by a step's weight phase)
  bool theta_pre = false;      // Theta of the current W already formed (a batch's grouped launch)
  int in_batch = 0;            // batches holding this walker set: their graphs bake its buffer addresses
  DevBuf logdet, logdet_new;   // nw x 2 complex
  DevBuf sing;                 // nw x 2 int
  DevBuf theta;                // nw x M x ntot complex
  DevBuf bpack, bpack_lo;      // packed B operand, both spins
  DevBuf tro, troo;            // nw x 2 x X complex: tr Omega, tr Omega^2
  DevBuf e1;                   // nw complex
  DevBuf eloc, parts, vbar;    // nw complex, nw x 3 complex, nw x X complex
  DevBuf coef;                 // nw x X complex (f64 or f32)
  DevBuf lfac;                 // nw: (Re log of the importance factor without the ratio, background phase)
  DevBuf amat;                 // nw x M x M complex (f64 or f32)
  DevBuf t1, t2;               // Taylor terms (nw x M x ntot, f64 or f32)
  DevBuf u;                    // Taylor sum (nw x M x ntot c128)
  DevBuf fields;               // nw x X f64 (device Philox)
  DevBuf gram, rinv;           // QR scratch (nw x 2 x n^2)
  DevBuf emix_tmp;             // scalar scratch
  size_t scratch_prec = (size_t)-1;
  // multi-determinant scratch
  DevBuf msd_tv;               // nw x msd_nv x ntot complex: C_V^H Theta
  DevBuf msd_d0[2];            // nw x n_exc complex: det A per spin
  DevBuf msd_S[2];             // nw x n_exc complex: sum over the excitation's determinants of conj(c) R(other spin)
  DevBuf msd_omega;            // (X + 1) msd_nr x chunk ntot complex: [C_ref^H; C_V^H] L^g Theta
  DevBuf msd_num;              // nw x (2 X + 1) complex: numerators (force bias, two-body per g, one-body)
  DevBuf msd_den;              // nw complex: sum_I conj(c_I) det A_I(up) det A_I(down)
  DevBuf msd_parts, msd_vbar;  // nw x 3 and nw x X complex: E1, E2, 0 and the force bias
  int msd_chunk = 0;           // walkers per Omega chunk
  // k-point scratch
  DevBuf kp_part;              // nw x 2 x nk x xq x nk x 3 complex: per-row-block traces
  DevBuf kp_cd;                // 2 x nw x nk xq complex: c and conj(d) of A = sum c L + d L^+
  DevBuf kp_tmp;               // 2 x nk x nw x nk m^2 complex: A-build GEMM outputs
  // FP32 ring scratch: packed coefficient rows, packed Theta-hat rows, force-bias partial tiles
  DevBuf r32_coef, r32_theta, r32_part;
  DevBuf r32_x;                // real form of A_w, packed for the Taylor products (FP32, or BF16 hi / lo planes)
  DevBuf r32_y[3];             // packed Taylor terms: V (FP32), then two alternating Horner terms
  int r32_layout = 0;          // layout r32_x / r32_y[1..2] were last cleared for: 1 FP32, 2 + t split BF16
                               // with product tile t
  DevBuf r32_b1w;              // walker rows (n, Re|Im) packed for the B1 products
  // four-index exchange scratch
  DevBuf eri_theta;            // packed Theta-hat hi / lo planes of one spin
  DevBuf eri_part;             // BF16x3: per (work unit, column) complex partial sums;
                               // FP64: Z^T = Theta-hat^T W'' rows of one spin (nw x N M complex)
  DevBuf eri_wg[2];            // BF16x3: (work unit, column block) of every workgroup of the launch
  std::vector<int> eri_wg_host[2];
  int eri_wg_launch[2] = {0, 0};
  long eri_wg_key[2] = {-1, -1};   // (units generation, column blocks) the layout was built for
};

// ---------------------------------------------------------------------------
// kernel launchers (all on the given stream)
// ---------------------------------------------------------------------------
enum GemmOp { OP_N = 0, OP_T = 1, OP_C = 2, OP_R = 3 };   // N, transpose, conj-transpose, conj

template <typename T> struct GemmArgs {
  int m, n, k, batch;
  const T* A; long lda, sA; int opA; bool cA;   // cA: A is complex (interleaved)
  const T* B; long ldb, sB; int opB; bool cB;
  T* C; long ldc, sC; bool cC;                  // cC: C complex
  double ar, ai, br, bi;                        // alpha, beta
  double2* D; long ldd, sD;                     // optional D += result (complex f64)
  // vn > 0: the n columns are batch members of vn columns each (column j is
  // column j % vn of member j / vn, at the member strides sB, sC, sD); batch = 1
  int vn;
};
// C = alpha op(A) op(B) + beta C   (D += alpha op(A) op(B) if D)
template <typename T> int gemm(const GemmArgs<T>& g, hipStream_t st);
template <typename T> GemmArgs<T> gemm_args();
void gemm_release_workspace(hipStream_t st);   // frees the split-k workspace of a stream

// batched in-place Gauss-Jordan inverse with partial pivoting of n x n complex
// matrices (stride between matrices `stride` elements). Writes inv (may be
// NULL: log det only), logdet (complex, per matrix), sing flag per matrix.
int lu_inverse(const double2* S, long stride, int n, int batch, double2* inv,
               double2* logdet, long ld_logdet, int* sing, long ld_sing, hipStream_t st);
// One deferred lu_inverse call (a batch of matrices of one system and spin).
struct GjTask {
  const double2* S;
  double2* inv;
  double2* logdet;
  int* sing;
  int stride, n, batch, ld_logdet, ld_sing;
};
// While a sink is installed on the calling thread, lu_inverse records its work
// there instead of launching it; lu_inverse_grouped then runs all recorded
// tasks of one register-block layout in one launch (the batch of many systems).
void lu_defer(std::vector<GjTask>* sink);
int lu_inverse_grouped(const std::vector<GjTask>& tasks, hipStream_t st);
// Cholesky of Hermitian G = R^H R then R^-1 (upper); logdet gets log det R (real part).
int chol_inverse(const double2* G, long stride, int n, int batch, double2* rinv,
                 double2* logdet, long ld_logdet, int* sing, long ld_sing, hipStream_t st);

int launch_fields(uint64_t seed, uint32_t sys_id, uint64_t step, int nw, int X, double* out,
                  long ld_step, int n_steps, hipStream_t st);

// system preparation
int system_prepare_dt(afq_system s, double dt);
int system_prepare_pack(afq_system s, int prec);

// walker pieces
int walkers_alloc_scratch(afq_walkers w);
int compute_overlap_theta(afq_system s, afq_walkers w, const double2* Wsrc, bool want_theta,
                          double2* logdet_out);
// one walker step; the Philox step index is *w->d_counter + step_off (the
// counter itself is advanced by counter_add after the steps of a call)
// coef_record (optional): where conj of this step's propagator coefficients go
int step_once(afq_system s, afq_walkers w, double dt, const double* fields, uint64_t seed,
              uint32_t sys_id, uint64_t step_off, bool do_qr, double e_shift, int order,
              double* emix_out, double* eloc_out, double* weights_out, double* ratio_out,
              void* coef_record = nullptr);
int step_stage(int stage, afq_system s, afq_walkers w, double dt, const double* fields, uint64_t seed,
              uint32_t sys_id, uint64_t step_off, bool do_qr, double e_shift, int order,
              double* emix_out, double* eloc_out, double* weights_out, double* ratio_out,
              void* coef_record = nullptr);
// Wout = B1 T_K(A) B1 Win with A_w = sum_n coef[w][n] L^n (coef in the system's contraction precision)
int propagate_walkers(afq_system s, afq_walkers w, int order, const void* coef, const double2* Win, double2* Wout);
// CholeskyQR2 of every spin block: src -> mid -> dst
int qr_orbitals(afq_system s, afq_walkers w, const double2* src, double2* mid, double2* dst);
// back-propagation window (bp.hip)
int bp_begin(afq_walkers w, int n_bp);
void bp_end(afq_walkers w);
void* bp_record_slot(afq_walkers w);   // NULL when the step is not recorded
int bp_check_step(afq_walkers w, int n_steps, double dt, int order);
void bp_advance(afq_walkers w, int n_steps);
int bp_comb_gather(afq_walkers w, const int* src);
int bp_rdm1(afq_walkers w, int qr_every, double* rdm_out, double* wsum_out);
int counter_add(uint64_t* c, uint64_t v, hipStream_t st);
int counter_set(uint64_t* c, uint64_t v, hipStream_t st);
int energy_backward(afq_system s, afq_walkers w, double scale, double* d_h1, double* d_chol,
                    double* d_walkers);

// exchange contraction: tr Omega and tr Omega^2 per (w, spin, n)
int exchange_launch(afq_system s, afq_walkers w, int spin, hipStream_t st);
int exchange_autotune(afq_system s, afq_walkers w, int reps, int* choice);   // choice[2]
int walkers_comb(afq_walkers w, double xi, int* src_out, double* total_out);
int pack_theta(afq_system s, afq_walkers w, hipStream_t st);

// k-point-blocked Cholesky (kpoint.hip)
int kp_system_create_impl(afq_system* out, int nk, const int32_t* kq, int m, int nu, int nd, int xq,
                          const double* hk, const double* Lk, const double* phik, double e_core, int prec,
                          void* stream);
int kp_prepare_dt(afq_system s, double dt);
// tr(L G^s), tr(L^+ G^s) and tr(Omega Omega') per (walker, spin, vector) -> tro / troo in the 2X-field layout
int kp_energy_traces(afq_system s, afq_walkers w, hipStream_t st);
// amat = sum_g (c_g L^g + d_g L^g+) from the 2X propagator coefficients coef (complex f64)
int kp_abuild(afq_system s, afq_walkers w, const double2* coef, hipStream_t st);

// FP32 ring contractions (ring32.hip)
int r32_prepare(afq_system s);                     // packed L (reduced modes) and Lt (split-BF16x3, real trial)
int r32_alloc_scratch(afq_system s, afq_walkers w);
bool r32_coulomb_used(afq_system s);
int b3_tile_of(afq_system s);       // the split-BF16x3 Taylor / B1 product tile a system uses
int b3_num_tiles();
int system_set_b3_tile(afq_system s, int tile);
int r32_autotune(afq_system s, afq_walkers w, int reps, int* tile_out);
bool r32_taylor_used(afq_system s);
// A_w = sum_n coef[w][n] L^n, written in packed real form to w->r32_x
int r32_abuild(afq_system s, afq_walkers w, const float* coef, hipStream_t st);
// w->u <- sum_{j <= order} A_w^j u / j! (Horner form, A_w from r32_abuild);
// with b1_rows, where the products can, the last one also writes u as the
// walker rows of the B1 product (*b1_rows tells whether it did)
int r32_taylor(afq_system s, afq_walkers w, int order, hipStream_t st, bool terms_packed = false,
               bool* b1_rows = nullptr);
// (B1 - I) packed for the current B1 (no-op when up to date)
int r32_prepare_b1(afq_system s);
// out = B1 in = in + (B1 - I) in for every walker (M x n_tot complex FP64 each);
// in_rows_packed: the split-BF16 walker rows of `in` are already in place
int r32_b1(afq_system s, afq_walkers w, const double2* in, double2* out, hipStream_t st, bool pack_terms = false,
           bool in_rows_packed = false);
// whether r32_b1(..., pack_terms = true) writes V in the packed term layouts of r32_taylor
bool r32_b1_packs_terms(afq_system s);
// tro[w][spin][n] = tr(Lt^{n,spin} Theta^spin) from the FP32 operands
int r32_coulomb(afq_system s, afq_walkers w, hipStream_t st);

// four-index exchange (eri.hip)
// builds or frees the W'' planes to match the system's precision, trial and form
int system_set_background(afq_system s, int on, const double* vmf);
int eri_sync(afq_system s);
int eri_alloc_scratch(afq_system s, afq_walkers w);
size_t eri_tensor_bytes(afq_system s);
// Theta-hat planes of one spin; then troo[w][spin][0] = sum_n tr(Omega_n Omega_n), troo[w][spin][n > 0] = 0
int eri_pack(afq_system s, afq_walkers w, int sp, hipStream_t st);
int eri_exchange(afq_system s, afq_walkers w, int sp, hipStream_t st);

// orthogonal multi-determinant trial (msd.hip)
constexpr int MSD_KMAX = 4;                                   // excitation rank per spin
constexpr int MSD_EXC = 1 + 3 * MSD_KMAX;                     // ints per device excitation record
int msd_set(afq_system s, const double* C, int n_det, const double* coeffs, const int32_t* exc);
int msd_alloc_scratch(afq_system s, afq_walkers w);
// energy pieces at the walkers whose Theta and log det are current: adds log(sum_I conj(c) R_I)
// to logdet[2w], writes msd_parts / msd_vbar
int msd_energy(afq_system s, afq_walkers w, double2* logdet, hipStream_t st);
// overlap correction only (Theta of the walkers in w->theta): logdet[2w] += log(sum_I conj(c) R_I)
int msd_overlap(afq_system s, afq_walkers w, double2* logdet, hipStream_t st);

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }
inline int round_up(int a, int b) { return (a + b - 1) / b * b; }
