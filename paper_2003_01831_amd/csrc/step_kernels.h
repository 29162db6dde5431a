// Launchers of the per-walker and elementwise kernels (step_kernels.hip).
#pragma once
#include "common.h"

struct AssembleArgs {
  int nw, ntot, M, X;
  const double2* thetaT;   // nw x ntot x M
  const double2* ht;       // ntot x M
  const double2* tro;      // nw x 2 x X
  const double2* troo;     // nw x 2 x X
  double e_core, dt;
  double fb_cap;           // force-bias modulus cap (0: off)
  const double* fields;    // nw x X or NULL (Philox)
  uint64_t seed;
  const uint64_t* step_ptr;  // device step counter; Philox step = *step_ptr + step_off
  uint64_t step_off;
  uint32_t sys_id;
  double2* eloc;           // nw (internal)
  double2* eloc_out;       // nw (optional, caller)
  double2* parts;          // nw x 3 (optional)
  double2* vbar_out;       // nw x X (optional)
  double2* lfac;           // nw (when coefficients are produced): (Re of sum_n x xbar - xbar^2/2 plus the
                           // background's c-number and constant, Im of the c-number = phase of the ratio)
  const double* vmf;       // X background c_n (mean-field subtraction) or NULL
  const double2* parts_in; // nw x 3 (E1, EJ, EK) given instead of computed (multi-determinant trial)
  const double2* vbar_in;  // nw x X force bias given with parts_in
};

struct WeightArgs {
  const double2* logdet_new;  // nw x 2
  const double2* logdet_cur;  // nw x 2
  const int* sing_new;        // nw x 2
  const double2* lfac;        // nw
  double* weights;            // nw
  int* alive;                 // nw
  int64_t* killed;            // 1
  double dt, e_shift;
  double w_cap;               // weight cap (0: off)
  double2* ratio_out;         // nw (optional)
  double* weights_out;        // nw (optional)
  double2* W;                 // nw x per
  const double2* Wn;          // nw x per
  long per;
  // optional: with W also copy S^-1 (sinv_per elements per walker) and the log
  // det of the propagated walkers (sinv_new, logdet_new -> sinv, logdet_keep)
  double2* sinv;
  const double2* sinv_new;
  double2* logdet_keep;
  long sinv_per;
  // 1: the caller has exchanged the buffers (W now holds W', Wn the old W;
  // sinv the new S^-1, sinv_new the old): only the walkers that died are
  // restored from the old buffers, instead of the live ones copied
  int swapped;
};

int pack_a(int prec, const double2* Lt, int X, int ntot, int M, int off, const PackShape& ps, bool real_trial,
           void* hi, void* lo, hipStream_t st);
int pack_b(int prec, const double2* thT, int nw, int ntot, int M, int off, const PackShape& ps, bool real_trial,
           void* hi, void* lo, hipStream_t st);
int convert_d2f(const double* x, float* y, long n, hipStream_t st);
int copy_d(const double* x, double* y, long n, hipStream_t st);
int real_part(const double2* z, double* y, long n, hipStream_t st);
// y[c][i] = Re z[i][c] for a rows x cols complex matrix
int fill_d(double* y, double v, long n, hipStream_t st);
int fill_i(int* y, int v, long n, hipStream_t st);
int fill_eye(double* y, int M, hipStream_t st);
int broadcast_trial(const double2* phi, double2* W, long per, int nw, hipStream_t st);
int masked_copy(const double2* src, double2* dst, long per, int nw, const int* alive, hipStream_t st,
                bool where_alive = true);
int launch_assemble(const AssembleArgs& a, void* coef, bool coef_f32, hipStream_t st);
int launch_emix(const double2* eloc, const double* wt, int nw, double* out, hipStream_t st);
int launch_weights(const WeightArgs& a, int nw, hipStream_t st);
// population control: comb indices (running sums in walker order, one thread),
// then the gather of the chosen walkers into Wout and the equal new weights
int launch_comb_index(const double* weights, int nw, double xi, double* cum, int* src, double* out2, hipStream_t st);
int launch_comb_apply(const double2* W, double2* Wout, long per, int nw, const int* src, const double* out2,
                      double* weights, int* alive, hipStream_t st);
int launch_asym(const double* x, int M, long nmat, double* out2, hipStream_t st);
int launch_maximag(const double2* z, long n, double* out, hipStream_t st);
int launch_infnorm(const double* x, int M, double* out, hipStream_t st);
int launch_logovlp(const double2* ld, int nw, double2* out, hipStream_t st);
int launch_init_alive(const double* wt, const int* sing, int nw, int* alive, int* bad, hipStream_t st);
// back-propagation window: conjugated coefficient copy, row gather (comb
// ancestry), weight sum + singular count, and the operands of the 1-RDM GEMM
int launch_conj_copy(const void* src, void* dst, long n, bool f32, hipStream_t st);
int launch_gather_rows(const void* src, void* dst, long row_bytes, int nrows, int nslabs, const int* idx,
                       hipStream_t st);
int launch_bp_stats(const double* wt, const int* sing, int nw, double* stats, hipStream_t st);
int launch_bp_pack(double2* Y, double2* Q, const double2* psi, long per, int ntot, int off, int n, int nw, int M,
                   const double* wt, const double* stats, hipStream_t st);
// Overlaps S^s_w = T^sH W^s_w of both spins in one launch (overlap.hip): T as
// phir (Re T, [M][ntot], real trial) or phi ([M][ntot] complex); S (w, s) at
// S + (2 w + s) nm2, row-major n_s x n_s. n_s <= 128.
int overlap_mfma(const double2* W, const double* phir, const double2* phi, int M, int ntot, int nw, const int n[2],
                 const int off[2], double2* S, long nm2, hipStream_t st);
// thetaT[w][off_s + b][k] = sum_j Sinv_ws[j][b] W[w][k][off_s + j], both spins in one launch
int theta_mfma(const double2* W, const double2* Sinv, int M, int ntot, int nw, const int n[2], const int off[2],
               long nm2, double2* thetaT, hipStream_t st);
// CholeskyQR products (overlap.hip), both spins in one launch each: the Gram
// matrices G_ws = W_ws^H W_ws (G laid out as S above) and Q_ws = W_ws Rinv_ws
// (Rinv as S^-1 above; Q in the walker layout, not W itself)
int gram_mfma(const double2* W, int M, int ntot, int nw, const int n[2], const int off[2], double2* G, long nm2,
              hipStream_t st);
int qr_apply_mfma(const double2* W, const double2* Rinv, int M, int ntot, int nw, const int n[2], const int off[2],
                  long nm2, double2* Q, hipStream_t st);
// Grouped launches of many walker sets (systems of a batch), one per
// electron-block count (and trial kind or wave count), each walking a work
// table. While an overlap sink is installed on the calling thread,
// overlap_mfma records its work there instead of launching it.
struct OvlTask {
  const double2* W;
  const double* phir;
  const double2* phi;
  double2* S;
  long nm2;
  int M, ntot, nw;
  int n[2], off[2];
};
void overlap_defer(std::vector<OvlTask>* sink);
int overlap_grouped(const std::vector<OvlTask>& tasks, hipStream_t st);
struct ThetaTask {
  const double2* W;
  const double2* Sinv;
  double2* thetaT;
  long nm2;
  int M, ntot, nw;
  int n[2], off[2];
};
int theta_grouped(const std::vector<ThetaTask>& tasks, hipStream_t st);
// the Theta product of a walker set's current walkers as such a task (walk.hip)
ThetaTask theta_task_of(afq_system s, afq_walkers w);
