// Walker objects and the sequence of one walker step:
//   overlap S = T^H W, S^-1 and log det S (FP64)  ->  Theta^T = S^-T W^T
//   -> packed Theta -> exchange/Coulomb traces -> E_L, force bias and the
//   propagator coefficients -> A = sum_n c_n L^n -> W' = B1 T_K(A) B1 W
//   -> new overlap and phaseless weight -> periodic CholeskyQR2.
#include "common.h"
#include "step_kernels.h"
#include "trace.h"

static size_t esz_of(int prec) { return prec == AFQ_FP64 ? 8 : prec == AFQ_CFP32 ? 4 : 2; }

int walkers_alloc_scratch(afq_walkers w) {
  afq_system s = w->sys;
  AFQ_RET(eri_alloc_scratch(s, w));
  AFQ_RET(r32_alloc_scratch(s, w));
  if (w->scratch_prec == (size_t)s->prec) return AFQ_OK;
  if (w->scratch_prec != (size_t)-1) w->exch_var[0] = w->exch_var[1] = -1;   // tuned for another precision
  const int nw = w->nw, M = s->M, ntot = s->ntot, X = s->X;
  const int nmax = std::max(s->n_up, s->n_dn);
  const size_t per = (size_t)M * ntot;
  const bool f64 = s->prec == AFQ_FP64;
  const size_t cz = f64 ? 16 : 8;  // complex element of the reduced-precision buffers
  if (!w->S.p) {
    AFQ_RET(w->S.alloc((size_t)nw * 2 * nmax * nmax * 16));
    AFQ_RET(w->Sinv.alloc((size_t)nw * 2 * nmax * nmax * 16));
    AFQ_RET(w->Sinv_new.alloc((size_t)nw * 2 * nmax * nmax * 16));
    AFQ_RET(w->logdet.alloc((size_t)nw * 2 * 16));
    AFQ_RET(w->logdet_new.alloc((size_t)nw * 2 * 16));
    AFQ_RET(w->sing.alloc((size_t)nw * 2 * sizeof(int)));
    AFQ_RET(w->theta.alloc((size_t)nw * per * 16));
    AFQ_RET(w->tro.alloc((size_t)nw * 2 * X * 16));
    AFQ_RET(w->troo.alloc((size_t)nw * 2 * X * 16));
    AFQ_RET(w->eloc.alloc((size_t)nw * 16));
    AFQ_RET(w->lfac.alloc((size_t)nw * 16));
    AFQ_RET(w->u.alloc((size_t)nw * per * 16));
    AFQ_RET(w->gram.alloc((size_t)nw * 2 * nmax * nmax * 16));
    AFQ_RET(w->rinv.alloc((size_t)nw * 2 * nmax * nmax * 16));
    AFQ_RET(w->emix_tmp.alloc(64));
  }
  size_t bsz = 0;
  for (int sp = 0; sp < 2; ++sp) bsz += (size_t)s->ps[sp].rows_b(nw) * s->ps[sp].kp;
  AFQ_RET(w->bpack.alloc(bsz * esz_of(s->prec)));
  if (s->prec == AFQ_BF16X3) AFQ_RET(w->bpack_lo.alloc(bsz * esz_of(s->prec)));
  else w->bpack_lo.free();
  AFQ_RET(w->coef.alloc((size_t)nw * X * cz));
  if (r32_taylor_used(s)) {   // the FP32 ring propagator keeps its own packed operands
    w->amat.free();
    w->t1.free();
    w->t2.free();
  } else {
    AFQ_RET(w->amat.alloc((size_t)nw * M * M * cz));
    AFQ_RET(w->t1.alloc((size_t)nw * per * cz));
    AFQ_RET(w->t2.alloc((size_t)nw * per * cz));
  }
  w->scratch_prec = (size_t)s->prec;
  return AFQ_OK;
}

// S^s = T^sH W^s for every walker (both spins, one launch); S^-1 into inv
// (optional) and log det
static int overlap_inverse(afq_system s, afq_walkers w, const double2* Wsrc, double2* inv, double2* logdet_out) {
  hipStream_t st = s->stream;
  const int nw = w->nw;
  const int nmax = std::max(s->n_up, s->n_dn);
  const long nm2 = (long)nmax * nmax;
  const int n[2] = {s->nspin_n(0), s->nspin_n(1)}, off[2] = {s->spin_off(0), s->spin_off(1)};
  AFQ_RET(overlap_mfma(Wsrc, s->phir.p ? s->phir.as<double>() : nullptr, s->phi.as<double2>(), s->M, s->ntot, nw,
                       n, off, w->S.as<double2>(), nm2, st));
  for (int sp = 0; sp < 2; ++sp)
    AFQ_RET(lu_inverse(w->S.as<double2>() + sp * nm2, 2 * nm2, n[sp], nw, inv ? inv + sp * nm2 : nullptr,
                       logdet_out + sp, 2, w->sing.as<int>() + sp, 2, st));
  return AFQ_OK;
}

// Theta^T from w->Sinv: thetaT[w][off + b][k] = sum_j (S^-1)[j][b] W[k][off + j]
static int theta_from_inverse(afq_system s, afq_walkers w, const double2* Wsrc) {
  const int nmax = std::max(s->n_up, s->n_dn);
  const int n[2] = {s->nspin_n(0), s->nspin_n(1)}, off[2] = {s->spin_off(0), s->spin_off(1)};
  return theta_mfma(Wsrc, w->Sinv.as<double2>(), s->M, s->ntot, w->nw, n, off, (long)nmax * nmax,
                    w->theta.as<double2>(), s->stream);
}

// the Theta product of the current walkers as a task of a grouped launch
ThetaTask theta_task_of(afq_system s, afq_walkers w) {
  const int nmax = std::max(s->n_up, s->n_dn);
  ThetaTask t{};
  t.W = w->W.as<double2>();
  t.Sinv = w->Sinv.as<double2>();
  t.thetaT = w->theta.as<double2>();
  t.nm2 = (long)nmax * nmax;
  t.M = s->M;
  t.ntot = s->ntot;
  t.nw = w->nw;
  for (int sp = 0; sp < 2; ++sp) {
    t.n[sp] = s->nspin_n(sp);
    t.off[sp] = s->spin_off(sp);
  }
  return t;
}

// S^s = T^sH W^s for every walker; S^-1 (optional) and log det; Theta^T = S^-T W^T
int compute_overlap_theta(afq_system s, afq_walkers w, const double2* Wsrc, bool want_theta, double2* logdet_out) {
  AFQ_RET(overlap_inverse(s, w, Wsrc, want_theta ? w->Sinv.as<double2>() : nullptr, logdet_out));
  if (want_theta) AFQ_RET(theta_from_inverse(s, w, Wsrc));
  return AFQ_OK;
}

int pack_theta(afq_system s, afq_walkers w, hipStream_t st) {
  const size_t esz = esz_of(s->prec);
  size_t off_bytes = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const PackShape& ps = s->ps[sp];
    void* hi = w->bpack.as<char>() + off_bytes;
    void* lo = s->prec == AFQ_BF16X3 ? (void*)(w->bpack_lo.as<char>() + off_bytes) : nullptr;
    AFQ_RET(pack_b(s->prec, w->theta.as<double2>(), w->nw, s->ntot, s->M, s->spin_off(sp), ps, s->real_trial, hi,
                   lo, st));
    off_bytes += (size_t)ps.rows_b(w->nw) * ps.kp * esz;
  }
  return AFQ_OK;
}

// Force bias / Coulomb traces in FP64: tro[w][s][n] = tr(Lt^{ns} Theta^s_w)
//   = sum_{(a,k)} thetaT[w][off + a][k] Lt[n][off + a][k]
// as one GEMM [nw x N M] x [N M x X] per spin. In split-BF16x3 mode this
// replaces the exchange kernel's traces: vbar enters EJ squared and the
// propagator, and its O(X N M) cost is 1/N of the exchange.
static int coulomb_fp64(afq_system s, afq_walkers w, hipStream_t st) {
  const int M = s->M, ntot = s->ntot, X = s->X;
  for (int sp = 0; sp < 2; ++sp) {
    const int n = s->nspin_n(sp), off = s->spin_off(sp);
    GemmArgs<double> g = gemm_args<double>();
    g.m = w->nw; g.n = X; g.k = n * M;
    g.A = w->theta.as<double>() + 2 * (long)off * M; g.lda = (long)ntot * M; g.cA = true;
    if (s->real_trial) {   // real half-rotated Cholesky rows: two real MFMAs per element
      g.B = s->LtRe.as<double>() + (long)off * M; g.ldb = (long)ntot * M; g.opB = OP_T; g.cB = false;
    } else {
      g.B = s->Lt.as<double>() + 2 * (long)off * M; g.ldb = (long)ntot * M; g.opB = OP_T; g.cB = true;
    }
    g.C = w->tro.as<double>() + 2 * (long)sp * X; g.ldc = 2L * X; g.cC = true;
    AFQ_RET(gemm<double>(g, st));
  }
  return AFQ_OK;
}

// Theta (already computed) -> exchange traces -> assembly (coef optional).
// With a multi-determinant trial the determinant sums replace the traces and
// log(sum_I conj(c_I) R_I) is added to logdet (the current walkers' log det).
static int energy_from_theta(afq_system s, afq_walkers w, AssembleArgs& a, bool want_coef, double2* logdet) {
  hipStream_t st = s->stream;
  if (s->kp_nk > 0) {
    TraceScope t(AFQ_PH_EXCHANGE, st);
    AFQ_RET(kp_energy_traces(s, w, st));
  } else if (s->msd_n > 0) {
    AFQ_RET(msd_energy(s, w, logdet, st));
    a.parts_in = w->msd_parts.as<double2>();
    a.vbar_in = w->msd_vbar.as<double2>();
  } else if (s->eri_ready) {   // four-index exchange (both spins in one launch when they share the tensor)
    for (int sp = 0; sp < (s->eri_share ? 1 : 2); ++sp) {
      {
        TraceScope t(AFQ_PH_PACK, st);
        AFQ_RET(eri_pack(s, w, sp, st));
      }
      TraceScope t(AFQ_PH_EXCHANGE, st);
      AFQ_RET(eri_exchange(s, w, sp, st));
    }
    TraceScope t(AFQ_PH_COULOMB, st);
    AFQ_RET(r32_coulomb_used(s) ? r32_coulomb(s, w, st) : coulomb_fp64(s, w, st));
  } else {
    {
      TraceScope t(AFQ_PH_PACK, st);
      AFQ_RET(pack_theta(s, w, st));
    }
    for (int sp = 0; sp < 2; ++sp) {
      TraceScope t(AFQ_PH_EXCHANGE, st);
      AFQ_RET(exchange_launch(s, w, sp, st));
    }
    if (s->prec == AFQ_BF16X3) {
      TraceScope t(AFQ_PH_COULOMB, st);
      AFQ_RET(r32_coulomb_used(s) ? r32_coulomb(s, w, st) : coulomb_fp64(s, w, st));
    }
  }
  TraceScope t(AFQ_PH_ASSEMBLE, st);
  a.nw = w->nw; a.ntot = s->ntot; a.M = s->M; a.X = s->X;
  a.thetaT = w->theta.as<double2>();
  a.ht = s->ht.as<double2>();
  a.tro = w->tro.as<double2>();
  a.troo = w->troo.as<double2>();
  a.e_core = s->e_core;
  a.eloc = w->eloc.as<double2>();
  a.lfac = want_coef ? w->lfac.as<double2>() : nullptr;
  return launch_assemble(a, want_coef ? w->coef.p : nullptr, s->prec != AFQ_FP64, st);
}

int energy_call(afq_system s, afq_walkers w, double* eloc_out, double* parts_out, double* vbar_out, double* emix_out) {
  AFQ_RET(system_prepare_pack(s, s->prec));
  AFQ_RET(walkers_alloc_scratch(w));
  AFQ_RET(compute_overlap_theta(s, w, w->W.as<double2>(), true, w->logdet.as<double2>()));
  AssembleArgs a{};
  a.dt = 0.0;
  a.eloc_out = reinterpret_cast<double2*>(eloc_out);
  a.parts = reinterpret_cast<double2*>(parts_out);
  a.vbar_out = reinterpret_cast<double2*>(vbar_out);
  AFQ_RET(energy_from_theta(s, w, a, false, w->logdet.as<double2>()));
  if (emix_out) AFQ_RET(launch_emix(w->eloc.as<double2>(), w->weights.as<double>(), w->nw, emix_out, s->stream));
  return AFQ_OK;
}

// Wout = B1 T_K(A) B1 Win for all walkers (complex A per walker, both spins at
// once), A_w = sum_n coef[w][n] L^n with coef in the contraction precision T.
template <typename T>
static int propagate(afq_system s, afq_walkers w, int order, const T* coef, const double2* Win, double2* Wout) {
  hipStream_t st = s->stream;
  const int M = s->M, ntot = s->ntot, nw = w->nw, X = s->X;
  const long per = (long)M * ntot;
  // A_w = sum_n c_wn L^n : [nw x X] (complex) x [X x M^2] (real)
  if (s->kp_nk > 0) {
    TraceScope tr(AFQ_PH_ABUILD, st);
    AFQ_RET(kp_abuild(s, w, reinterpret_cast<const double2*>(coef), st));
  } else if (sizeof(T) == 4 && r32_taylor_used(s)) {   // reduced modes: the FP32 ring contraction
    TraceScope tr(AFQ_PH_ABUILD, st);
    AFQ_RET(r32_abuild(s, w, reinterpret_cast<const float*>(coef), st));
  } else {
    TraceScope tr(AFQ_PH_ABUILD, st);
    GemmArgs<T> g = gemm_args<T>();
    g.m = nw; g.n = M * M; g.k = X;
    g.A = coef; g.lda = X; g.cA = true;
    g.B = reinterpret_cast<const T*>(s->chol.p);
    g.ldb = (long)M * M; g.cB = false;
    g.C = w->amat.as<T>(); g.ldc = (long)M * M; g.cC = true;
    AFQ_RET(gemm<T>(g, st));
  }
  TraceScope tr(AFQ_PH_TAYLOR, st);
  const bool ring = sizeof(T) == 4 && s->kp_nk == 0 && r32_taylor_used(s);
  bool u_rows = false;   // the last Taylor product also wrote U as the B1 product's walker rows
  // U = B1 W  (FP64; the walkers' columns side by side as one n = nw ntot product)
  if (ring) {   // reduced modes: W + (B1 - I) W with the correction on the FP32 ring
    AFQ_RET(r32_b1(s, w, Win, w->u.as<double2>(), st, true));   // also packs V for the Taylor products where it can
  } else {
    GemmArgs<double> g = gemm_args<double>();
    g.m = M; g.n = nw * ntot; g.k = M; g.vn = ntot;
    g.A = s->kp_nk ? s->B1c.as<double>() : s->B1.as<double>(); g.lda = M; g.cA = s->kp_nk > 0; g.sA = 0;
    g.B = reinterpret_cast<const double*>(Win); g.ldb = ntot; g.cB = true; g.sB = per;
    g.C = w->u.as<double>(); g.ldc = ntot; g.cC = true; g.sC = per;
    AFQ_RET(gemm<double>(g, st));
  }
  if (ring) {
    // reduced modes: U <- T_K(A) U in Horner form on the FP32 ring kernel
    AFQ_RET(r32_taylor(s, w, order, st, r32_b1_packs_terms(s), &u_rows));
  } else {
    // term_0 = U (in the contraction precision); term_j = A term_{j-1} / j; U += term_j
    T* cur = w->t1.as<T>();
    T* nxt = w->t2.as<T>();
    if (sizeof(T) == 8) AFQ_RET(copy_d(w->u.as<double>(), reinterpret_cast<double*>(cur), 2 * per * nw, st));
    else AFQ_RET(convert_d2f(w->u.as<double>(), reinterpret_cast<float*>(cur), 2 * per * nw, st));
    for (int j = 1; j <= order; ++j) {
      GemmArgs<T> g = gemm_args<T>();
      g.m = M; g.n = ntot; g.k = M; g.batch = nw;
      g.A = w->amat.as<T>(); g.lda = M; g.cA = true; g.sA = (long)M * M;
      g.B = cur; g.ldb = ntot; g.cB = true; g.sB = per;
      g.C = j < order ? nxt : nullptr; g.ldc = ntot; g.cC = true; g.sC = per;
      g.ar = 1.0 / j;
      g.D = w->u.as<double2>(); g.ldd = ntot; g.sD = per;
      AFQ_RET(gemm<T>(g, st));
      std::swap(cur, nxt);
    }
  }
  // W' = B1 U
  if (ring) {
    AFQ_RET(r32_b1(s, w, w->u.as<double2>(), Wout, st, false, u_rows));
  } else {
    GemmArgs<double> g = gemm_args<double>();
    g.m = M; g.n = nw * ntot; g.k = M; g.vn = ntot;
    g.A = s->kp_nk ? s->B1c.as<double>() : s->B1.as<double>(); g.lda = M; g.cA = s->kp_nk > 0; g.sA = 0;
    g.B = w->u.as<double>(); g.ldb = ntot; g.cB = true; g.sB = per;
    g.C = reinterpret_cast<double*>(Wout); g.ldc = ntot; g.cC = true; g.sC = per;
    AFQ_RET(gemm<double>(g, st));
  }
  return AFQ_OK;
}

int propagate_walkers(afq_system s, afq_walkers w, int order, const void* coef, const double2* Win, double2* Wout) {
  if (s->prec == AFQ_FP64) return propagate<double>(s, w, order, static_cast<const double*>(coef), Win, Wout);
  return propagate<float>(s, w, order, static_cast<const float*>(coef), Win, Wout);
}

// CholeskyQR of every spin block of every walker (positive diagonal R). FP64
// mode runs two passes, dst^s = (src^s R1^-1) R2^-1 with the first written to
// mid (all three nw x M x ntot complex), so that Q is orthonormal to FP64
// rounding whatever the conditioning. The reduced modes run one pass: its
// loss of orthogonality, about cond(W)^2 times the FP64 unit roundoff, is far
// below their own rounding for walkers re-orthonormalised every few steps, and
// the step depends on W only through its column span.
int qr_orbitals(afq_system s, afq_walkers w, const double2* src0, double2* mid, double2* dst0) {
  hipStream_t st = s->stream;
  const int M = s->M, ntot = s->ntot, nw = w->nw;
  const int nmax = std::max(s->n_up, s->n_dn);
  const long nm2 = (long)nmax * nmax;
  const int npass = s->prec == AFQ_FP64 ? 2 : 1;
  const double2* in[2] = {src0, mid};
  double2* out[2] = {npass == 2 ? mid : dst0, dst0};
  const int n[2] = {s->nspin_n(0), s->nspin_n(1)}, off[2] = {s->spin_off(0), s->spin_off(1)};
  for (int pass = 0; pass < npass; ++pass) {
    AFQ_RET(gram_mfma(in[pass], M, ntot, nw, n, off, w->gram.as<double2>(), nm2, st));
    for (int sp = 0; sp < 2; ++sp)
      AFQ_RET(chol_inverse(w->gram.as<double2>() + sp * nm2, 2 * nm2, n[sp], nw, w->rinv.as<double2>() + sp * nm2,
                           w->logdet_new.as<double2>() + sp, 2, w->sing.as<int>() + sp, 2, st));
    AFQ_RET(qr_apply_mfma(in[pass], w->rinv.as<double2>(), M, ntot, nw, n, off, nm2, out[pass], st));
  }
  return AFQ_OK;
}

// QR of the live walkers: W -> Wn -> u, then u back into W where alive (for
// a walker set outside any batch: the buffers exchanged, the walkers not
// alive given their old W back)
static int qr_walkers(afq_system s, afq_walkers w) {
  w->s_carried = false;   // W changes
  TraceScope tr(AFQ_PH_QR, s->stream);
  AFQ_RET(qr_orbitals(s, w, w->W.as<double2>(), w->Wn.as<double2>(), w->u.as<double2>()));
  const long per = (long)s->M * s->ntot;
  if (w->in_batch == 0) {
    w->W.swap(w->u);
    return masked_copy(w->u.as<double2>(), w->W.as<double2>(), per, w->nw, w->alive.as<int>(), s->stream, false);
  }
  return masked_copy(w->u.as<double2>(), w->W.as<double2>(), per, w->nw, w->alive.as<int>(), s->stream);
}

// One step in three stages that end where an overlap inverse is needed: stage
// 0 forms S = T^H W (when S^-1 was not carried over) and requests its inverse;
// stage 1 forms Theta, the energy, the propagated walkers and S' = T^H W' and
// requests its inverse (or log det); stage 2 applies the phaseless weight and
// QR. step_once runs them back to back; a batch of systems runs each stage on
// every system and the requested inverses of all systems as grouped launches
// in between (lu_defer).
int step_stage(int stage, afq_system s, afq_walkers w, double dt, const double* fields, uint64_t seed,
               uint32_t sys_id, uint64_t step_off, bool do_qr, double e_shift, int order, double* emix_out,
               double* eloc_out, double* weights_out, double* ratio_out, void* coef_record) {
  hipStream_t st = s->stream;
  const int nw = w->nw;
  // with QR at the end of the step (or a multi-determinant trial) the new
  // overlap's inverse is not carried to the next step
  const bool carry = s->msd_n == 0 && !do_qr;
  if (stage == 0) {
    // S^-1 and log det are still those the previous step's weight phase
    // carried over with W unless something has changed W since
    TraceScope t(AFQ_PH_OVERLAP, st);
    if (!w->s_carried || s->msd_n > 0)   // a multi-determinant trial leaves its own overlap in logdet
      AFQ_RET(overlap_inverse(s, w, w->W.as<double2>(), w->Sinv.as<double2>(), w->logdet.as<double2>()));
    return AFQ_OK;
  }
  if (stage == 1) {
    if (w->theta_pre) {   // formed by a batch's grouped launch before this stage
      w->theta_pre = false;
    } else {
      TraceScope t(AFQ_PH_OVERLAP, st);
      AFQ_RET(theta_from_inverse(s, w, w->W.as<double2>()));
    }
    AssembleArgs a{};
    a.dt = dt;
    a.fields = fields;
    a.seed = seed;
    a.step_ptr = w->d_counter.as<uint64_t>();
    a.step_off = step_off;
    a.sys_id = sys_id;
    a.fb_cap = w->fb_cap;
    a.vmf = s->mf_on ? s->vmf.as<double>() : nullptr;
    a.eloc_out = reinterpret_cast<double2*>(eloc_out);
    AFQ_RET(energy_from_theta(s, w, a, true, w->logdet.as<double2>()));
    if (coef_record)   // back-propagation window: conj(c) of this step, the coefficients of B^H
      AFQ_RET(launch_conj_copy(w->coef.p, coef_record, (long)nw * s->X, s->prec != AFQ_FP64, st));
    if (emix_out) {
      TraceScope t(AFQ_PH_ASSEMBLE, st);
      AFQ_RET(launch_emix(w->eloc.as<double2>(), w->weights.as<double>(), nw, emix_out, st));
    }
    AFQ_RET(propagate_walkers(s, w, order, w->coef.p, w->W.as<double2>(), w->Wn.as<double2>()));
    // new overlap: its full inverse when it is carried to the next step with
    // the walkers the weight kernel keeps (hardly dearer than its determinant),
    // or with a multi-determinant trial (whose Theta of W' the ratio needs)
    TraceScope tw(AFQ_PH_WEIGHT, st);
    const bool want_inv = carry || s->msd_n > 0;
    return overlap_inverse(s, w, w->Wn.as<double2>(),
                           want_inv ? (carry ? w->Sinv_new.as<double2>() : w->Sinv.as<double2>()) : nullptr,
                           w->logdet_new.as<double2>());
  }
  {
    TraceScope tw(AFQ_PH_WEIGHT, st);
    if (s->msd_n > 0) {
      AFQ_RET(theta_from_inverse(s, w, w->Wn.as<double2>()));
      AFQ_RET(msd_overlap(s, w, w->logdet_new.as<double2>(), st));
    }
    WeightArgs wa{};
    wa.logdet_new = w->logdet_new.as<double2>();
    wa.logdet_cur = w->logdet.as<double2>();
    wa.sing_new = w->sing.as<int>();
    wa.lfac = w->lfac.as<double2>();
    wa.weights = w->weights.as<double>();
    wa.alive = w->alive.as<int>();
    wa.killed = w->killed.as<int64_t>();
    wa.dt = dt;
    wa.e_shift = e_shift;
    wa.w_cap = w->w_cap;
    wa.ratio_out = reinterpret_cast<double2*>(ratio_out);
    wa.weights_out = weights_out;
    // A walker set outside any batch takes W' (and the new S^-1) by exchanging
    // the buffers, and only the walkers that died get their old values back;
    // a batch's captured graph holds the buffer addresses, so there the live
    // walkers are copied instead
    if (w->in_batch == 0) {
      w->W.swap(w->Wn);
      if (carry) w->Sinv.swap(w->Sinv_new);
      wa.swapped = 1;
    }
    wa.W = w->W.as<double2>();
    wa.Wn = w->Wn.as<double2>();
    wa.per = (long)s->M * s->ntot;
    if (carry) {
      const int nmax = std::max(s->n_up, s->n_dn);
      wa.sinv = w->Sinv.as<double2>();
      wa.sinv_new = w->Sinv_new.as<double2>();
      wa.logdet_keep = w->logdet.as<double2>();
      wa.sinv_per = 2L * nmax * nmax;
    }
    AFQ_RET(launch_weights(wa, nw, st));
  }
  w->s_carried = carry;
  if (do_qr) AFQ_RET(qr_walkers(s, w));
  return AFQ_OK;
}

int step_once(afq_system s, afq_walkers w, double dt, const double* fields, uint64_t seed, uint32_t sys_id,
              uint64_t step_off, bool do_qr, double e_shift, int order, double* emix_out, double* eloc_out,
              double* weights_out, double* ratio_out, void* coef_record) {
  for (int stage = 0; stage < 3; ++stage)
    AFQ_RET(step_stage(stage, s, w, dt, fields, seed, sys_id, step_off, do_qr, e_shift, order, emix_out, eloc_out,
                       weights_out, ratio_out, coef_record));
  return AFQ_OK;
}

int walkers_create_impl(afq_walkers* out, afq_system s, int nw, const double* w0, const double* wt0) {
  AFQ_CHECK(out, AFQ_E_INVALID, "afq_walkers_create: out is NULL");
  *out = nullptr;
  AFQ_CHECK(s, AFQ_E_INVALID, "afq_walkers_create: system is NULL");
  AFQ_CHECK(nw >= 1 && nw <= 65535, AFQ_E_INVALID, "afq_walkers_create: n_walkers must be in [1, 65535]");
  afq_walkers w = new afq_walkers_s();
  int rc = [&]() -> int {
    w->sys = s;
    w->nw = nw;
    hipStream_t st = s->stream;
    const long per = (long)s->M * s->ntot;
    AFQ_RET(w->W.alloc((size_t)nw * per * 16));
    AFQ_RET(w->Wn.alloc((size_t)nw * per * 16));
    AFQ_RET(w->weights.alloc((size_t)nw * 8));
    AFQ_RET(w->alive.alloc((size_t)nw * 4));
    AFQ_RET(w->killed.alloc(16));
    AFQ_TRY_HIP(hipMemsetAsync(w->killed.p, 0, 16, st));
    AFQ_RET(w->d_counter.alloc(sizeof(uint64_t)));
    AFQ_RET(counter_set(w->d_counter.as<uint64_t>(), 0, st));
    if (w0) AFQ_TRY_HIP(hipMemcpyAsync(w->W.p, w0, (size_t)nw * per * 16, hipMemcpyDeviceToDevice, st));
    else AFQ_RET(broadcast_trial(s->phi.as<double2>(), w->W.as<double2>(), per, nw, st));
    if (wt0) AFQ_TRY_HIP(hipMemcpyAsync(w->weights.p, wt0, (size_t)nw * 8, hipMemcpyDeviceToDevice, st));
    else AFQ_RET(fill_d(w->weights.as<double>(), 1.0, nw, st));
    AFQ_RET(walkers_alloc_scratch(w));
    AFQ_RET(compute_overlap_theta(s, w, w->W.as<double2>(), false, w->logdet.as<double2>()));
    int* bad = reinterpret_cast<int*>(w->emix_tmp.p);
    AFQ_TRY_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    AFQ_RET(launch_init_alive(w->weights.as<double>(), w->sing.as<int>(), nw, w->alive.as<int>(), bad, st));
    int hbad = 0;
    AFQ_TRY_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    AFQ_TRY_HIP(hipStreamSynchronize(st));
    AFQ_CHECK(hbad == 0, AFQ_E_SINGULAR, "afq_walkers_create: a live walker has a singular overlap with the trial");
    return AFQ_OK;
  }();
  if (rc != AFQ_OK) {
    delete w;
    return rc;
  }
  *out = w;
  return AFQ_OK;
}

// Population control: comb the walkers to nw copies of equal weight (see
// comb_index_kernel). Synchronises the stream to read the total weight back.
int walkers_comb(afq_walkers w, double xi, int* src_out, double* total_out) {
  afq_system s = w->sys;
  hipStream_t st = s->stream;
  const int nw = w->nw;
  AFQ_RET(w->comb_cum.alloc((size_t)nw * sizeof(double)));
  AFQ_RET(w->comb_src.alloc((size_t)nw * sizeof(int)));
  AFQ_RET(w->comb_out.alloc(2 * sizeof(double)));
  AFQ_RET(launch_comb_index(w->weights.as<double>(), nw, xi, w->comb_cum.as<double>(), w->comb_src.as<int>(),
                            w->comb_out.as<double>(), st));
  double out2[2];
  AFQ_TRY_HIP(hipMemcpyAsync(out2, w->comb_out.p, sizeof(out2), hipMemcpyDeviceToHost, st));
  AFQ_TRY_HIP(hipStreamSynchronize(st));
  if (total_out) *total_out = out2[0];
  AFQ_CHECK(out2[0] > 0.0 && std::isfinite(out2[0]), AFQ_E_STATE,
            "afq_walkers_comb: the walkers carry no positive weight");
  const long per = (long)s->M * s->ntot;
  AFQ_RET(launch_comb_apply(w->W.as<double2>(), w->Wn.as<double2>(), per, nw, w->comb_src.as<int>(),
                            w->comb_out.as<double>(), w->weights.as<double>(), w->alive.as<int>(), st));
  AFQ_TRY_HIP(hipMemcpyAsync(w->W.p, w->Wn.p, (size_t)nw * per * 16, hipMemcpyDeviceToDevice, st));
  w->s_carried = false;
  AFQ_RET(bp_comb_gather(w, w->comb_src.as<int>()));
  if (src_out) {
    AFQ_TRY_HIP(hipMemcpyAsync(src_out, w->comb_src.p, (size_t)nw * sizeof(int), hipMemcpyDeviceToHost, st));
    AFQ_TRY_HIP(hipStreamSynchronize(st));
  }
  return AFQ_OK;
}
