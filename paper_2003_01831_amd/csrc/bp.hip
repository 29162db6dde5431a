// Back-propagated one-body density matrix (back-propagation paragraph of the
// AFQMC section). A window opens on the current walkers phi_w (kept as the
// kets); each of the next n steps stores conj(c) of every walker's propagator
// coefficients. The estimator then carries the trial backwards,
//   |psi_w> = B_0^H B_1^H ... B_{n-1}^H |T>,   B_j^H = B1 T_K(A_j^H) B1,
// A_j^H = sum_n conj(c_jn) L^n (L^n and B1 real symmetric; the Taylor
// polynomial of A^H is the adjoint of that of A), so the same batched
// propagator as the walk runs on the bras with the stored coefficients in
// reverse order. With the weights w_w at the end of the window,
//   P^s_ij = sum_w w_w <psi_w| c+_is c_js |phi_w> / <psi_w|phi_w> / sum_w w_w
//          = sum_w f_w (phi_w^s (psi_w^sH phi_w^s)^-1 psi_w^sH)_ji,
// which is one GEMM over the walker-stacked index: P^s = Q Y^T with
// Q[i][(w, a)] = conj(psi_w[i][a]) and Y[j][(w, a)] = f_w (phi_w S_w^-1)[j][a].
// A comb inside the window hands every copy its source walker's ket and
// stored coefficients (row gathers with the comb's source indices).
#include <cmath>
#include "common.h"
#include "step_kernels.h"
#include "trace.h"

static size_t coef_elem(int prec) { return prec == AFQ_FP64 ? 16 : 8; }

static int ensure(DevBuf& b, size_t n) { return b.bytes >= n && b.p ? AFQ_OK : b.alloc(n); }

int bp_begin(afq_walkers w, int n_bp) {
  afq_system s = w->sys;
  hipStream_t st = s->stream;
  const size_t per = (size_t)s->M * s->ntot;
  w->bp_n = -1;
  AFQ_RET(ensure(w->bp_W0, (size_t)w->nw * per * 16));
  const size_t cb = (size_t)n_bp * w->nw * s->X * coef_elem(s->prec);
  if (cb > 0) AFQ_RET(ensure(w->bp_coef, cb));
  AFQ_TRY_HIP(hipMemcpyAsync(w->bp_W0.p, w->W.p, (size_t)w->nw * per * 16, hipMemcpyDeviceToDevice, st));
  w->bp_n = n_bp;
  w->bp_rec = 0;
  w->bp_start = w->counter;
  w->bp_dt = -1.0;
  w->bp_order = 0;
  w->bp_prec = s->prec;
  w->bp_b1 = s->b1_serial;
  return AFQ_OK;
}

void bp_end(afq_walkers w) {
  w->bp_n = -1;
  w->bp_W0.free();
  w->bp_coef.free();
  w->bp_tmp.free();
  w->bp_psi.free();
  w->bp_stats.free();
}

// validation before n_steps steps of an afq_step call; the first recorded step
// fixes dt and the Taylor order of the window
int bp_check_step(afq_walkers w, int n_steps, double dt, int order) {
  if (w->bp_n < 0 || w->bp_rec >= w->bp_n || n_steps == 0) return AFQ_OK;
  AFQ_CHECK(w->sys->prec == w->bp_prec, AFQ_E_STATE,
            "afq_step: the precision changed while a back-propagation window records");
  AFQ_CHECK(w->sys->b1_serial == w->bp_b1, AFQ_E_STATE,
            "afq_step: the background subtraction changed while a back-propagation window records");
  if (w->bp_rec > 0) {
    AFQ_CHECK(dt == w->bp_dt && order == w->bp_order, AFQ_E_INVALID,
              "afq_step: dt and the Taylor order must stay fixed while a back-propagation window records");
  } else {
    w->bp_dt = dt;
    w->bp_order = order;
  }
  return AFQ_OK;
}

void* bp_record_slot(afq_walkers w) {
  if (w->bp_n < 0 || w->bp_rec >= w->bp_n) return nullptr;
  const size_t slot = (size_t)w->nw * w->sys->X * coef_elem(w->bp_prec);
  return w->bp_coef.as<char>() + (size_t)w->bp_rec * slot;
}

void bp_advance(afq_walkers w, int n_steps) {
  if (w->bp_n >= 0) w->bp_rec = std::min(w->bp_n, w->bp_rec + n_steps);
}

// after a comb (src = device source indices): gather kets and stored rows
int bp_comb_gather(afq_walkers w, const int* src) {
  if (w->bp_n < 0) return AFQ_OK;
  afq_system s = w->sys;
  hipStream_t st = s->stream;
  const size_t per = (size_t)s->M * s->ntot;
  AFQ_RET(launch_gather_rows(w->bp_W0.p, w->Wn.p, (long)per * 16, w->nw, 1, src, st));
  AFQ_TRY_HIP(hipMemcpyAsync(w->bp_W0.p, w->Wn.p, (size_t)w->nw * per * 16, hipMemcpyDeviceToDevice, st));
  if (w->bp_rec > 0) {
    const long row = (long)s->X * coef_elem(w->bp_prec);
    AFQ_RET(ensure(w->bp_tmp, w->bp_coef.bytes));
    AFQ_RET(launch_gather_rows(w->bp_coef.p, w->bp_tmp.p, row, w->nw, w->bp_rec, src, st));
    std::swap(w->bp_coef.p, w->bp_tmp.p);
    std::swap(w->bp_coef.bytes, w->bp_tmp.bytes);
  }
  return AFQ_OK;
}

int bp_rdm1(afq_walkers w, int qr_every, double* rdm_out, double* wsum_out) {
  w->s_carried = false;   // S, S^-1 and the log dets are scratch here
  afq_system s = w->sys;
  AFQ_CHECK(w->bp_n >= 0, AFQ_E_STATE, "afq_bp_rdm1: no back-propagation window is open");
  AFQ_CHECK(w->bp_rec == w->bp_n, AFQ_E_STATE,
            "afq_bp_rdm1: the window has recorded " + std::to_string(w->bp_rec) + " of its " +
                std::to_string(w->bp_n) + " steps");
  AFQ_CHECK(w->counter == w->bp_start + (uint64_t)w->bp_n, AFQ_E_STATE,
            "afq_bp_rdm1: steps were taken after the window filled (the weights must be those at its end)");
  AFQ_CHECK(s->prec == w->bp_prec, AFQ_E_STATE, "afq_bp_rdm1: the precision changed since the window opened");
  AFQ_CHECK(s->b1_serial == w->bp_b1, AFQ_E_STATE,
            "afq_bp_rdm1: the background subtraction changed since the window opened");
  hipStream_t st = s->stream;
  const int M = s->M, ntot = s->ntot, nw = w->nw, X = s->X;
  const long per = (long)M * ntot;
  const int nmax = std::max(s->n_up, s->n_dn);
  const long nm2 = (long)nmax * nmax;
  if (w->bp_n > 0) AFQ_RET(system_prepare_dt(s, w->bp_dt));
  AFQ_RET(system_prepare_pack(s, s->prec));
  AFQ_RET(walkers_alloc_scratch(w));
  AFQ_RET(ensure(w->bp_psi, (size_t)nw * per * 16));
  AFQ_RET(ensure(w->bp_stats, 2 * sizeof(double)));

  // bras: B_{n-1}^H acts first on the trial
  double2* cur = w->bp_psi.as<double2>();
  double2* oth = w->Wn.as<double2>();
  AFQ_RET(broadcast_trial(s->phi.as<double2>(), cur, per, nw, st));
  const size_t slot = (size_t)nw * X * coef_elem(w->bp_prec);
  for (int t = 0; t < w->bp_n; ++t) {
    const int j = w->bp_n - 1 - t;
    AFQ_RET(propagate_walkers(s, w, w->bp_order, w->bp_coef.as<char>() + (size_t)j * slot, cur, oth));
    std::swap(cur, oth);
    if (qr_every > 0 && (t + 1) % qr_every == 0) {
      TraceScope tr(AFQ_PH_QR, st);
      AFQ_RET(qr_orbitals(s, w, cur, w->theta.as<double2>(), oth));
      std::swap(cur, oth);
    }
  }

  // S^s_w = psi_w^sH phi_w^s and its inverse, both spins
  const double* kets = w->bp_W0.as<double>();
  for (int sp = 0; sp < 2; ++sp) {
    const int n = s->nspin_n(sp), off = s->spin_off(sp);
    GemmArgs<double> g = gemm_args<double>();
    g.m = n; g.n = n; g.k = M; g.batch = nw;
    g.A = reinterpret_cast<const double*>(cur) + 2 * off; g.lda = ntot; g.opA = OP_C; g.cA = true; g.sA = per;
    g.B = kets + 2 * off; g.ldb = ntot; g.cB = true; g.sB = per;
    g.C = w->S.as<double>() + 2 * sp * nm2; g.ldc = n; g.cC = true; g.sC = 2 * nm2;
    AFQ_RET(gemm<double>(g, st));
    AFQ_RET(lu_inverse(w->S.as<double2>() + sp * nm2, 2 * nm2, n, nw, w->Sinv.as<double2>() + sp * nm2,
                       w->logdet_new.as<double2>() + sp, 2, w->sing.as<int>() + sp, 2, st));
  }
  AFQ_RET(launch_bp_stats(w->weights.as<double>(), w->sing.as<int>(), nw, w->bp_stats.as<double>(), st));

  // per spin: Y (theta) = phi S^-1 stacked over walkers, Q (u) = conj(psi), P^s = Q Y^T
  long stack = 0;   // complex offset of this spin's operands in theta and u
  for (int sp = 0; sp < 2; ++sp) {
    const int n = s->nspin_n(sp), off = s->spin_off(sp);
    const long K = (long)nw * n;
    double2* Y = w->theta.as<double2>() + stack;
    double2* Q = w->u.as<double2>() + stack;
    GemmArgs<double> y = gemm_args<double>();
    y.m = M; y.n = n; y.k = n; y.batch = nw;
    y.A = kets + 2 * off; y.lda = ntot; y.cA = true; y.sA = per;
    y.B = w->Sinv.as<double>() + 2 * sp * nm2; y.ldb = n; y.cB = true; y.sB = 2 * nm2;
    y.C = reinterpret_cast<double*>(Y); y.ldc = K; y.cC = true; y.sC = n;
    AFQ_RET(gemm<double>(y, st));
    AFQ_RET(launch_bp_pack(Y, Q, cur, per, ntot, off, n, nw, M, w->weights.as<double>(), w->bp_stats.as<double>(),
                           st));
    GemmArgs<double> p = gemm_args<double>();
    p.m = M; p.n = M; p.k = (int)K; p.batch = 1;
    p.A = reinterpret_cast<const double*>(Q); p.lda = K; p.cA = true;
    p.B = reinterpret_cast<const double*>(Y); p.ldb = K; p.opB = OP_T; p.cB = true;
    p.C = rdm_out + 2L * sp * M * M; p.ldc = M; p.cC = true;
    AFQ_RET(gemm<double>(p, st));
    stack += (long)M * K;
  }
  double stats[2];
  AFQ_TRY_HIP(hipMemcpyAsync(stats, w->bp_stats.p, sizeof(stats), hipMemcpyDeviceToHost, st));
  AFQ_TRY_HIP(hipStreamSynchronize(st));
  if (wsum_out) *wsum_out = stats[0];
  AFQ_CHECK(stats[0] > 0.0 && std::isfinite(stats[0]), AFQ_E_STATE, "afq_bp_rdm1: no walker has positive weight");
  AFQ_CHECK(stats[1] == 0.0, AFQ_E_SINGULAR,
            "afq_bp_rdm1: a walker of positive weight has a singular overlap with its back-propagated trial");
  return AFQ_OK;
}
