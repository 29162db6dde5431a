// k-point-blocked Cholesky factorisation (the explicitly k-point dependent
// factorisation of the AFQMC section and its row of Table tab:afqmc_comp).
//
// Orbitals (k, i), i < m, map to k m + i. Every (Q, n) is one complex
// Cholesky vector whose only non-zero blocks are (k + Q, k) = L^{Q,k}_n, so the
// two-electron tensor is the paper's v_ijkl = sum_g L^g_ik conj(L^g_lj) with
// non-Hermitian L^g. With a_g = (L + L^+)/2 and b_g = (L - L^+)/(2i):
//   H = sum h'_ik c+_i c_k + 1/2 sum_g (A_g^2 + B_g^2),
//   h' = h - 1/4 sum_g (L L^+ + L^+ L)   (block diagonal in k),
// two Hubbard-Stratonovich fields per vector (x for a_g, y for b_g), and
//   E_L = E_II + tr(h G) + 1/2 sum_g [tr(L G) tr(L^+ G) - sum_s tr(L G^s L^+ G^s)].
// The walkers are dense M x N (the fields couple all k-blocks); the trial is
// block diagonal (n orbitals per k-point and spin). What the blocks buy:
//  * A = sum_g (c_g L^g + d_g L^g+) is built from two GEMMs batched over Q
//    over the m x m blocks (x_c m^2 N_k^2 per walker instead of x_c N_k m^2 N_k^2),
//  * Omega = (T^H L^g) Theta has one non-zero block column per row block: for
//    row block k1 and vector (Q, n), Omega[k1, :] = Lt^{Q,k1-Q}_n Theta[k1-Q, :]
//    (n x m times m x N), and tr(Omega Omega') pairs it with
//    Omega'[k', k1] = Ltd^{Q,k'}_n Theta[k'+Q, k1] (Ltd = (T^k)^H (L^{Q,k})^+),
//    which are the batched per-(Q, k) contractions of cost x_c m^2 n^2 N_k^3.
// Everything runs in FP64. The field coefficients enter the common assembly
// kernel as 2 nk xq force biases (tr a G, tr b G): their squares sum to
// tr(L G) tr(L^+ G), and the exchange traces fill the first half of troo.
#include <algorithm>
#include <cmath>
#include <vector>
#include "common.h"
#include "step_kernels.h"
#include "trace.h"

constexpr size_t KP_MAX_LDS = 160 * 1024;

// ---------------------------------------------------------------------------
// host helpers (set-up only)
// ---------------------------------------------------------------------------
static void hmatmul(const double2* A, const double2* B, double2* C, int m) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double2 s = make_double2(0.0, 0.0);
      for (int k = 0; k < m; ++k) s = cadd(s, cmul(A[i * m + k], B[k * m + j]));
      C[i * m + j] = s;
    }
}

// exp(Z) of an m x m complex block: Z / 2^q with infinity norm <= 1/2, order-18
// Horner Taylor polynomial, q squarings
static void hexpm(const double2* Z, double2* E, int m) {
  double nrm = 0.0;
  for (int i = 0; i < m; ++i) {
    double r = 0.0;
    for (int j = 0; j < m; ++j) r += std::hypot(Z[i * m + j].x, Z[i * m + j].y);
    nrm = std::max(nrm, r);
  }
  int q = 0;
  while (nrm / std::ldexp(1.0, q) > 0.5 && q < 60) ++q;
  const double sc = 1.0 / std::ldexp(1.0, q);
  std::vector<double2> z((size_t)m * m), cur((size_t)m * m), nxt((size_t)m * m), t((size_t)m * m);
  for (size_t e = 0; e < z.size(); ++e) z[e] = cscale(Z[e], sc);
  auto eye = [&](std::vector<double2>& a) {
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) a[(size_t)i * m + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  };
  eye(cur);
  for (int j = 18; j >= 1; --j) {     // E_j = I + (z / j) E_{j+1}
    hmatmul(z.data(), cur.data(), t.data(), m);
    eye(nxt);
    for (size_t e = 0; e < t.size(); ++e) nxt[e] = cadd(nxt[e], cscale(t[e], 1.0 / j));
    std::swap(cur, nxt);
  }
  for (int i = 0; i < q; ++i) {
    hmatmul(cur.data(), cur.data(), t.data(), m);
    std::swap(cur, t);
  }
  std::copy(cur.begin(), cur.end(), E);
}

int kp_prepare_dt(afq_system s, double dt) {
  if (s->B1c.p && s->B1_dt == dt) return AFQ_OK;
  const int nk = s->kp_nk, m = s->kp_m, M = s->M;
  std::vector<double2> B((size_t)M * M, make_double2(0.0, 0.0)), z((size_t)m * m), e((size_t)m * m);
  for (int k = 0; k < nk; ++k) {
    for (size_t x = 0; x < z.size(); ++x) z[x] = cscale(s->kp_hp[(size_t)k * m * m + x], -0.5 * dt);
    hexpm(z.data(), e.data(), m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) B[(size_t)(k * m + i) * M + k * m + j] = e[(size_t)i * m + j];
  }
  if (!s->B1c.p) AFQ_RET(s->B1c.alloc(B.size() * 16));
  AFQ_TRY_HIP(hipMemcpyAsync(s->B1c.p, B.data(), B.size() * 16, hipMemcpyHostToDevice, s->stream));
  AFQ_TRY_HIP(hipStreamSynchronize(s->stream));
  s->B1_dt = dt;
  return AFQ_OK;
}

static size_t kp_lds_bytes(int nk, int m, int nmax, int xq) {
  const size_t N = (size_t)nk * nmax, M = (size_t)nk * m;
  return ((size_t)m * N + M * nmax + (size_t)nmax * m + (size_t)nk * nmax * m + (size_t)xq * 12) * 16;
}

int kp_system_create_impl(afq_system* out, int nk, const int32_t* kq, int m, int nu, int nd, int xq,
                          const double* hk, const double* Lk, const double* phik, double e_core, int prec,
                          void* stream) {
  AFQ_CHECK(out, AFQ_E_INVALID, "afq_kp_system_create: out is NULL");
  *out = nullptr;
  AFQ_CHECK(nk >= 1 && nk <= 64 && m >= 1 && xq >= 1, AFQ_E_INVALID,
            "afq_kp_system_create: need 1 <= nk <= 64, m >= 1, xq >= 1");
  AFQ_CHECK(nu >= 1 && nd >= 1 && nu <= m && nd <= m, AFQ_E_INVALID,
            "afq_kp_system_create: need 1 <= n_up, n_dn <= m per k-point");
  AFQ_CHECK((long)nk * m <= 4096 && (long)nk * std::max(nu, nd) <= 128, AFQ_E_UNSUPPORTED,
            "afq_kp_system_create: at most 4096 orbitals and 128 electrons per spin");
  AFQ_CHECK(kq && hk && Lk && phik, AFQ_E_INVALID, "afq_kp_system_create: NULL input");
  AFQ_CHECK(prec == AFQ_FP64, AFQ_E_UNSUPPORTED, "afq_kp_system_create: k-point systems run in FP64 mode");
  AFQ_CHECK(std::isfinite(e_core), AFQ_E_INVALID, "afq_kp_system_create: e_core is not finite");
  // the table must be an abelian group law with identity 0
  std::vector<int> kd((size_t)nk * nk, -1);
  for (int Q = 0; Q < nk; ++Q)
    for (int k = 0; k < nk; ++k) {
      const int v = kq[Q * nk + k];
      AFQ_CHECK(v >= 0 && v < nk, AFQ_E_INVALID, "afq_kp_system_create: k-point table entry out of range");
      AFQ_CHECK(v == kq[k * nk + Q], AFQ_E_INVALID, "afq_kp_system_create: k-point table is not symmetric");
      AFQ_CHECK(kd[(size_t)v * nk + k] < 0, AFQ_E_INVALID,
                "afq_kp_system_create: k-point table column is not a permutation");
      kd[(size_t)v * nk + k] = Q;
    }
  for (int k = 0; k < nk; ++k)
    AFQ_CHECK(kq[k] == k, AFQ_E_INVALID, "afq_kp_system_create: k-point 0 must be the identity");
  for (int a = 0; a < nk; ++a)
    for (int b = 0; b < nk; ++b)
      for (int c = 0; c < nk; ++c)
        AFQ_CHECK(kq[a * nk + kq[b * nk + c]] == kq[kq[a * nk + b] * nk + c], AFQ_E_INVALID,
                  "afq_kp_system_create: k-point table is not associative");
  const int M = nk * m, Nu = nk * nu, Nd = nk * nd, ntot = Nu + Nd, nkn = nu + nd;
  const size_t lds = kp_lds_bytes(nk, m, std::max(nu, nd), xq);
  AFQ_CHECK(lds <= KP_MAX_LDS, AFQ_E_UNSUPPORTED, "afq_kp_system_create: the trace kernel needs more than 160 KB of LDS");
  afq_system s = new afq_system_s();
  int rc = [&]() -> int {
    s->M = M; s->n_up = Nu; s->n_dn = Nd; s->ntot = ntot; s->X = 2 * nk * xq;
    s->e_core = e_core;
    s->stream = static_cast<hipStream_t>(stream);
    s->real_trial = false;
    s->kp_nk = nk; s->kp_m = m; s->kp_xq = xq; s->kp_nu = nu; s->kp_nd = nd;
    s->kp_lds = lds;
    AFQ_TRY_HIP(hipGetDevice(&s->device));
    hipStream_t st = s->stream;
    const size_t mm = (size_t)m * m, nL = (size_t)nk * nk * xq * mm;
    std::vector<double2> h((size_t)nk * mm), L(nL), ph((size_t)nk * m * nkn);
    AFQ_TRY_HIP(hipMemcpyAsync(h.data(), hk, h.size() * 16, hipMemcpyDeviceToHost, st));
    AFQ_TRY_HIP(hipMemcpyAsync(L.data(), Lk, L.size() * 16, hipMemcpyDeviceToHost, st));
    AFQ_TRY_HIP(hipMemcpyAsync(ph.data(), phik, ph.size() * 16, hipMemcpyDeviceToHost, st));
    AFQ_TRY_HIP(hipStreamSynchronize(st));
    // validation: Hermitian h^k, finite inputs
    double hmax = 0.0, hasym = 0.0;
    for (int k = 0; k < nk; ++k)
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          const double2 a = h[k * mm + i * m + j], b = h[k * mm + j * m + i];
          AFQ_CHECK(std::isfinite(a.x) && std::isfinite(a.y), AFQ_E_INVALID, "afq_kp_system_create: non-finite h");
          hmax = std::max(hmax, std::hypot(a.x, a.y));
          hasym = std::max(hasym, std::hypot(a.x - b.x, a.y + b.y));
        }
    AFQ_CHECK(hasym <= 1e-12 * hmax + 1e-300, AFQ_E_INVALID, "afq_kp_system_create: an h^k block is not Hermitian");
    for (const double2& v : L)
      AFQ_CHECK(std::isfinite(v.x) && std::isfinite(v.y), AFQ_E_INVALID,
                "afq_kp_system_create: non-finite Cholesky block");
    const auto Lb = [&](int Q, int k, int n) { return &L[(((size_t)Q * nk + k) * xq + n) * mm]; };
    // dense h and block-diagonal trial (columns: up (k, a) k-major, then down)
    std::vector<double2> hd((size_t)M * M, make_double2(0.0, 0.0)), T((size_t)M * ntot, make_double2(0.0, 0.0));
    for (int k = 0; k < nk; ++k)
      for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j) hd[(size_t)(k * m + i) * M + k * m + j] = h[k * mm + i * m + j];
        for (int a = 0; a < nu; ++a) T[(size_t)(k * m + i) * ntot + k * nu + a] = ph[((size_t)k * m + i) * nkn + a];
        for (int a = 0; a < nd; ++a)
          T[(size_t)(k * m + i) * ntot + Nu + k * nd + a] = ph[((size_t)k * m + i) * nkn + nu + a];
      }
    // h'^k = h^k - 1/4 sum_{Q,n} [L^{Q,k-Q} L^{Q,k-Q}+ + L^{Q,k}+ L^{Q,k}]
    s->kp_hp.assign((size_t)nk * mm, make_double2(0.0, 0.0));
    for (int k = 0; k < nk; ++k) {
      double2* hp = &s->kp_hp[(size_t)k * mm];
      for (size_t e = 0; e < mm; ++e) hp[e] = h[k * mm + e];
      for (int Q = 0; Q < nk; ++Q) {
        int ksrc = -1;                                         // the k' with k' + Q = k
        for (int c = 0; c < nk; ++c)
          if (kq[Q * nk + c] == k) ksrc = c;
        for (int n = 0; n < xq; ++n) {
          const double2* A = Lb(Q, ksrc, n);
          const double2* B = Lb(Q, k, n);
          for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
              double2 acc = make_double2(0.0, 0.0);
              for (int l = 0; l < m; ++l) {
                acc = cadd(acc, cmul(A[i * m + l], cconj(A[j * m + l])));     // (L L^+)_ij
                acc = cadd(acc, cmul(cconj(B[l * m + i]), B[l * m + j]));     // (L^+ L)_ij
              }
              hp[i * m + j] = csub(hp[i * m + j], cscale(acc, 0.25));
            }
        }
      }
    }
    // ht = T^H h (ntot x M)
    std::vector<double2> ht((size_t)ntot * M, make_double2(0.0, 0.0));
    for (int c = 0; c < ntot; ++c) {
      const int k = c < Nu ? c / nu : (c - Nu) / nd;
      for (int l = 0; l < m; ++l) {
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < m; ++i) acc = cadd(acc, cmul(cconj(T[(size_t)(k * m + i) * ntot + c]), h[k * mm + i * m + l]));
        ht[(size_t)c * M + k * m + l] = acc;
      }
    }
    // Lt[Q][k][n][a][l] = sum_i conj(T^{k+Q}[i][a]) L^{Q,k}_n[i][l];
    // Ltd[Q][k][n][a][l] = sum_i conj(T^k[i][a]) conj(L^{Q,k}_n[l][i]); a over the nu + nd trial columns of a k-point
    const size_t nLt = (size_t)nk * nk * xq * nkn * m;
    std::vector<double2> Lt(nLt), Ltd(nLt), Lr(nL);
    for (int Q = 0; Q < nk; ++Q)
      for (int k = 0; k < nk; ++k) {
        const int kk = kq[Q * nk + k];
        for (int n = 0; n < xq; ++n) {
          const double2* B = Lb(Q, k, n);
          double2* o = &Lt[(((size_t)Q * nk + k) * xq + n) * nkn * m];
          double2* od = &Ltd[(((size_t)Q * nk + k) * xq + n) * nkn * m];
          for (int a = 0; a < nkn; ++a)
            for (int l = 0; l < m; ++l) {
              double2 acc = make_double2(0.0, 0.0), accd = make_double2(0.0, 0.0);
              for (int i = 0; i < m; ++i) {
                acc = cadd(acc, cmul(cconj(ph[((size_t)kk * m + i) * nkn + a]), B[i * m + l]));
                accd = cadd(accd, cmul(cconj(ph[((size_t)k * m + i) * nkn + a]), cconj(B[l * m + i])));
              }
              o[a * m + l] = acc;
              od[a * m + l] = accd;
            }
          // [Q][n][k][i][l] for the A-build GEMMs
          std::copy(B, B + mm, &Lr[(((size_t)Q * xq + n) * nk + k) * mm]);
        }
      }
    AFQ_RET(s->phi.alloc(T.size() * 16));
    AFQ_RET(s->kp_h.alloc(hd.size() * 16));
    AFQ_RET(s->ht.alloc(ht.size() * 16));
    AFQ_RET(s->kp_Lt.alloc(nLt * 16));
    AFQ_RET(s->kp_Ltd.alloc(nLt * 16));
    AFQ_RET(s->kp_L.alloc(nL * 16));
    AFQ_RET(s->kp_kq.alloc((size_t)nk * nk * sizeof(int)));
    AFQ_RET(s->kp_kd.alloc((size_t)nk * nk * sizeof(int)));
    AFQ_TRY_HIP(hipMemcpyAsync(s->phi.p, T.data(), T.size() * 16, hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->kp_h.p, hd.data(), hd.size() * 16, hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->ht.p, ht.data(), ht.size() * 16, hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->kp_Lt.p, Lt.data(), nLt * 16, hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->kp_Ltd.p, Ltd.data(), nLt * 16, hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->kp_L.p, Lr.data(), nL * 16, hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->kp_kq.p, kq, (size_t)nk * nk * sizeof(int), hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->kp_kd.p, kd.data(), kd.size() * sizeof(int), hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipStreamSynchronize(st));
    s->prec = prec;
    s->apack_prec = prec;
    return AFQ_OK;
  }();
  if (rc != AFQ_OK) {
    delete s;
    return rc;
  }
  *out = s;
  return AFQ_OK;
}

// ---------------------------------------------------------------------------
// A-build: c_g = (coef_x - i coef_y)/2 and conj(d_g) = conj((coef_x + i coef_y)/2),
// then per Q two GEMMs over the blocks and one scatter into the dense A
// ---------------------------------------------------------------------------
__global__ void kp_cd_kernel(const double2* __restrict__ coef, int nw, int XL, double2* __restrict__ c,
                             double2* __restrict__ dbar) {
  const long total = (long)nw * XL;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long w = e / XL, g = e - w * XL;
    const double2 x = coef[w * 2 * XL + g], y = coef[w * 2 * XL + XL + g];
    c[e] = make_double2(0.5 * (x.x + y.y), 0.5 * (x.y - y.x));        // (x - i y)/2
    dbar[e] = make_double2(0.5 * (x.x - y.y), -0.5 * (x.y + y.x));    // conj((x + i y)/2)
  }
}

// A[w][(k1,i),(k2,l)] = tc[kd(k1,k2)][w][k2][i][l] + conj(td[kd(k2,k1)][w][k1][l][i])
__global__ void kp_scatter_kernel(const double2* __restrict__ tc, const double2* __restrict__ td,
                                  const int* __restrict__ kd, int nk, int m, int nw, double2* __restrict__ A) {
  const int M = nk * m;
  const long mm = (long)m * m, blk = (long)nk * mm, perQ = (long)nw * blk;
  const long total = (long)nw * M * M;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long w = e / ((long)M * M);
    const long r = e - w * M * M;
    const int row = (int)(r / M), col = (int)(r - (long)row * M);
    const int k1 = row / m, i = row - k1 * m, k2 = col / m, l = col - k2 * m;
    const int Q = kd[k1 * nk + k2], Qd = kd[k2 * nk + k1];
    const double2 a = tc[Q * perQ + w * blk + k2 * mm + i * m + l];
    const double2 b = td[Qd * perQ + w * blk + k1 * mm + l * m + i];
    A[e] = make_double2(a.x + b.x, a.y - b.y);
  }
}

static int grid_of(long total) { return (int)std::min<long>(std::max<long>(ceil_div(total, 256), 1), 65536); }

int kp_abuild(afq_system s, afq_walkers w, const double2* coef, hipStream_t st) {
  const int nk = s->kp_nk, m = s->kp_m, xq = s->kp_xq, nw = w->nw, XL = nk * xq;
  const long mm = (long)m * m, blk = (long)nk * mm;
  const size_t cd = (size_t)2 * nw * XL * 16, tmp = (size_t)2 * nk * nw * blk * 16;
  if (w->kp_cd.bytes < cd) AFQ_RET(w->kp_cd.alloc(cd));
  if (w->kp_tmp.bytes < tmp) AFQ_RET(w->kp_tmp.alloc(tmp));
  double2* c = w->kp_cd.as<double2>();
  double2* dbar = c + (size_t)nw * XL;
  hipLaunchKernelGGL(kp_cd_kernel, dim3(grid_of((long)nw * XL)), dim3(256), 0, st, coef, nw, XL, c, dbar);
  AFQ_TRY_HIP(hipGetLastError());
  double2* tc = w->kp_tmp.as<double2>();
  double2* td = tc + (size_t)nk * nw * blk;
  for (int part = 0; part < 2; ++part) {
    // t[Q][w][(k, i, l)] = sum_n coef[w][Q xq + n] L[Q][n][(k, i, l)]
    GemmArgs<double> g = gemm_args<double>();
    g.m = nw; g.n = (int)blk; g.k = xq; g.batch = nk;
    g.A = reinterpret_cast<const double*>(part ? dbar : c); g.lda = XL; g.cA = true; g.sA = xq;
    g.B = s->kp_L.as<double>(); g.ldb = blk; g.cB = true; g.sB = (long)xq * blk;
    g.C = reinterpret_cast<double*>(part ? td : tc); g.ldc = blk; g.cC = true; g.sC = (long)nw * blk;
    AFQ_RET(gemm<double>(g, st));
  }
  hipLaunchKernelGGL(kp_scatter_kernel, dim3(grid_of((long)nw * s->M * s->M)), dim3(256), 0, st, tc, td,
                     s->kp_kd.as<int>(), nk, m, nw, w->amat.as<double2>());
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// ---------------------------------------------------------------------------
// traces: one workgroup per (row block k1, Q, walker x spin). For every n:
//   Omega[(k1,a),(k',b)]  = sum_l Lt^{Q,k2}_n[a][l] Theta[(k2,l),(k',b)],   k2 + Q = k1
//   Omega'[(k',b),(k1,a)] = sum_l Ltd^{Q,k'}_n[b][l] Theta[(k'+Q,l),(k1,a)]
// and the row block's share of tr(Omega Omega'), tr(Omega), tr(Omega').
// ---------------------------------------------------------------------------
struct KpTraceArgs {
  const double2* thetaT;   // nw x ntot x M
  const double2* Lt;       // [Q][k][n][a][l], a over nkn = nu + nd
  const double2* Ltd;
  const int* kq;
  const int* kd;
  int nk, m, xq, nu, nd, ntot, M;
  double2* part;           // [w][spin][Q][n][k1][3]
};

__device__ inline double2 wave_sum(double2 v) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  return v;
}

__global__ __launch_bounds__(256) void kp_trace_kernel(KpTraceArgs a) {
  extern __shared__ double2 lds[];
  const int k1 = blockIdx.x, Q = blockIdx.y, w = blockIdx.z >> 1, sp = blockIdx.z & 1, t = threadIdx.x;
  const int nk = a.nk, m = a.m, M = a.M;
  const int ns = sp ? a.nd : a.nu, N = nk * ns, off = sp ? nk * a.nu : 0, aoff = sp ? a.nu : 0;
  const int nkn = a.nu + a.nd;
  int ksrc = 0;                                        // k2 with k2 + Q = k1
  for (int c = 0; c < nk; ++c)
    if (a.kq[Q * nk + c] == k1) ksrc = c;
  double2* thA = lds;                       // [l][c]: Theta[(ksrc, l), c], c < N
  double2* thB = thA + (long)m * N;         // [r][aa]: Theta[r, (k1, aa)], r < M, aa < ns
  double2* LtS = thB + (long)M * ns;        // [aa][l]: Lt^{Q,ksrc}_n
  double2* LtdS = LtS + (long)ns * m;       // [k'][b][l]: Ltd^{Q,k'}_n
  double2* wp = LtdS + (long)nk * ns * m;   // [n][wave][3]
  const double2* th = a.thetaT + (long)w * a.ntot * M;
  for (int e = t; e < N * m; e += 256) {
    const int c = e / m, l = e - c * m;
    thA[l * N + c] = th[(long)(off + c) * M + ksrc * m + l];
  }
  for (int e = t; e < ns * M; e += 256) {
    const int aa = e / M, r = e - aa * M;
    thB[r * ns + aa] = th[(long)(off + k1 * ns + aa) * M + r];
  }
  const int lane = t & 63, wave = t >> 6;
  const int npair = ns * N;                 // (aa, k', b)
  for (int n = 0; n < a.xq; ++n) {
    __syncthreads();                        // previous n done with LtS / LtdS; Theta staged
    const double2* lt = a.Lt + ((((long)Q * nk + ksrc) * a.xq + n) * nkn + aoff) * m;
    for (int e = t; e < ns * m; e += 256) LtS[e] = lt[e];
    for (int e = t; e < nk * ns * m; e += 256) {
      const int kp = e / (ns * m), rest = e - kp * ns * m;
      LtdS[e] = a.Ltd[((((long)Q * nk + kp) * a.xq + n) * nkn + aoff) * m + rest];
    }
    __syncthreads();
    double2 ek = make_double2(0.0, 0.0), tl = make_double2(0.0, 0.0), tld = make_double2(0.0, 0.0);
    for (int p = t; p < npair; p += 256) {
      const int aa = p / N, c = p - aa * N, kp = c / ns, b = c - kp * ns;
      const int rb = a.kq[Q * nk + kp];     // row block k' + Q of Theta for Omega'
      double2 om = make_double2(0.0, 0.0), omd = make_double2(0.0, 0.0);
      for (int l = 0; l < m; ++l) {
        om = cadd(om, cmul(LtS[aa * m + l], thA[l * N + c]));
        omd = cadd(omd, cmul(LtdS[(kp * ns + b) * m + l], thB[(rb * m + l) * ns + aa]));
      }
      ek = cadd(ek, cmul(om, omd));
      if (kp == k1 && aa == b) {
        tl = cadd(tl, om);
        tld = cadd(tld, omd);
      }
    }
    ek = wave_sum(ek);
    tl = wave_sum(tl);
    tld = wave_sum(tld);
    if (lane == 0) {
      wp[(n * 4 + wave) * 3] = ek;
      wp[(n * 4 + wave) * 3 + 1] = tl;
      wp[(n * 4 + wave) * 3 + 2] = tld;
    }
  }
  __syncthreads();
  double2* out = a.part + ((((long)w * 2 + sp) * nk + Q) * a.xq) * nk * 3;
  for (int e = t; e < a.xq * 3; e += 256) {
    const int n = e / 3, j = e - n * 3;
    double2 v = wp[(n * 4) * 3 + j];
    for (int q = 1; q < 4; ++q) v = cadd(v, wp[(n * 4 + q) * 3 + j]);
    out[((long)n * nk + k1) * 3 + j] = v;
  }
}

// per (walker, spin): sum the row blocks (fixed order) into the 2X-field layout
//   tro[g] = (tr L G + tr L^+ G)/2, tro[XL + g] = (tr L G - tr L^+ G)/(2i),
//   troo[g] = tr(Omega Omega'), troo[XL + g] = 0
__global__ void kp_reduce_kernel(const double2* __restrict__ part, int nk, int xq, double2* __restrict__ tro,
                                 double2* __restrict__ troo) {
  const int ws = blockIdx.y, XL = nk * xq;
  for (int g = blockIdx.x * 256 + threadIdx.x; g < XL; g += gridDim.x * 256) {
    const double2* p = part + ((long)ws * XL + g) * nk * 3;
    double2 ek = make_double2(0.0, 0.0), tl = make_double2(0.0, 0.0), tld = make_double2(0.0, 0.0);
    for (int k1 = 0; k1 < nk; ++k1) {
      ek = cadd(ek, p[k1 * 3]);
      tl = cadd(tl, p[k1 * 3 + 1]);
      tld = cadd(tld, p[k1 * 3 + 2]);
    }
    double2* o = tro + (long)ws * 2 * XL;
    double2* oo = troo + (long)ws * 2 * XL;
    o[g] = make_double2(0.5 * (tl.x + tld.x), 0.5 * (tl.y + tld.y));
    o[XL + g] = make_double2(0.5 * (tl.y - tld.y), -0.5 * (tl.x - tld.x));   // -i (tl - tld) / 2
    oo[g] = ek;
    oo[XL + g] = make_double2(0.0, 0.0);
  }
}

int kp_energy_traces(afq_system s, afq_walkers w, hipStream_t st) {
  const int nk = s->kp_nk, xq = s->kp_xq, nw = w->nw;
  const size_t part = (size_t)nw * 2 * nk * xq * nk * 3 * 16;
  if (w->kp_part.bytes < part) AFQ_RET(w->kp_part.alloc(part));
  static bool attr = false;
  if (s->kp_lds > 64 * 1024 && !attr) {
    AFQ_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kp_trace_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)KP_MAX_LDS));
    attr = true;
  }
  KpTraceArgs a{};
  a.thetaT = w->theta.as<double2>();
  a.Lt = s->kp_Lt.as<double2>();
  a.Ltd = s->kp_Ltd.as<double2>();
  a.kq = s->kp_kq.as<int>();
  a.kd = s->kp_kd.as<int>();
  a.nk = nk; a.m = s->kp_m; a.xq = xq; a.nu = s->kp_nu; a.nd = s->kp_nd; a.ntot = s->ntot; a.M = s->M;
  a.part = w->kp_part.as<double2>();
  hipLaunchKernelGGL(kp_trace_kernel, dim3(nk, nk, 2 * nw), dim3(256), s->kp_lds, st, a);
  AFQ_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(kp_reduce_kernel, dim3(ceil_div(nk * xq, 256), 2 * nw), dim3(256), 0, st, w->kp_part.as<double2>(),
                     nk, xq, w->tro.as<double2>(), w->troo.as<double2>());
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
