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
constexpr int KP_NS_MAX = 16;   // electrons per k-point and spin held in registers by the trace kernel

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

// dynamic LDS of the trace kernel: the larger of the two spins' layouts
// (Theta rows m x N, columns M x ns, the per-thread shares npar x N x 3, the
// per-vector sums xq x 3, one pass's Lt rows npar x ns x m; N = nk ns and
// npar = 256 / N vectors per pass, so a spin with fewer electrons can need more)
static size_t kp_lds_bytes(int nk, int m, int nu, int nd, int xq) {
  size_t need = 0;
  for (int ns : {nu, nd}) {
    if (ns < 1) continue;
    const size_t N = (size_t)nk * ns, M = (size_t)nk * m, npar = 256 / N;
    need = std::max(need, ((size_t)m * N + M * ns + npar * N * 3 + (size_t)xq * 3 + npar * ns * m) * 16);
  }
  return need;
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
  AFQ_CHECK(std::max(nu, nd) <= KP_NS_MAX && nk * std::max(nu, nd) <= 256, AFQ_E_UNSUPPORTED,
            "afq_kp_system_create: at most 16 electrons per k-point and spin");
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
  const size_t lds = kp_lds_bytes(nk, m, nu, nd, xq);
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
// traces: one workgroup per (row block k1, walker, Q) and spin; the workgroups
// running together share Q (Q is the slowest grid index), so the Lt and Ltd
// rows of that Q stay in L2 while the walkers go by. With k2 + Q = k1,
// for every vector n and every column c = (k', b) of the spin's trial block:
//   Omega[(k1,a), c]      = sum_l Lt^{Q,k2}_n[a][l]  Theta[(k2, l), c]
//   Omega'[c, (k1,a)]     = sum_l Ltd^{Q,k'}_n[b][l] Theta[(k'+Q, l), (k1, a)]
// One thread owns one (n, c) and all a: it keeps the 2 x ns accumulators, so
// each Theta / Ltd element it loads feeds ns multiply-adds. The Theta block
// rows (k2, .) and the columns (k1, .) are staged in LDS once per workgroup,
// the Lt rows of the pass's vectors (shared by the N threads of a vector) once
// per pass;
// the row block's shares of tr(Omega Omega'), tr(Omega), tr(Omega') are summed
// over the columns in a fixed order.
// ---------------------------------------------------------------------------
struct KpTraceArgs {
  const double2* thetaT;   // nw x ntot x M
  const double2* Lt;       // [Q][k][n][a][l], a over nkn = nu + nd
  const double2* Ltd;
  const int* kq;
  int nk, m, xq, nu, nd, ntot, M;
  double2* part;           // [w][spin][Q][n][k1][3]
};

template <int NS>
__global__ __launch_bounds__(256) void kp_trace_kernel(KpTraceArgs a, int sp) {
  extern __shared__ double2 lds[];
  const int k1 = blockIdx.x, w = blockIdx.y, Q = blockIdx.z, t = threadIdx.x;
  const int nk = a.nk, m = a.m, M = a.M;
  const int ns = NS, N = nk * ns, off = sp ? nk * a.nu : 0, aoff = sp ? a.nu : 0;
  const int nkn = a.nu + a.nd;
  int k2 = 0;                               // k2 + Q = k1
  for (int c = 0; c < nk; ++c)
    if (a.kq[Q * nk + c] == k1) k2 = c;
  const int npar = 256 / N;                 // vectors per pass
  double2* thA = lds;                       // [l][c]: Theta[(k2, l), c]
  double2* thB = thA + (long)m * N;         // [r][aa]: Theta[r, (k1, aa)]
  double2* pp = thB + (long)M * ns;         // [npar][N][3]: per-thread shares of one pass
  double2* wp = pp + (long)npar * N * 3;    // [xq][3]
  double2* ltb = wp + (long)a.xq * 3;       // [npar][a][l]: Lt^{Q,k2}_n of the pass's vectors
  const double2* th = a.thetaT + (long)w * a.ntot * M;
  for (int e = t; e < N * m; e += 256) {
    const int c = e / m, l = e - c * m;
    thA[l * N + c] = th[(long)(off + c) * M + k2 * m + l];
  }
  for (int e = t; e < ns * M; e += 256) {
    const int aa = e / M, r = e - aa * M;
    thB[r * ns + aa] = th[(long)(off + k1 * ns + aa) * M + r];
  }
  __syncthreads();
  const int nl = t / N, c = t - nl * N;
  const int kp = c / ns, b = c - kp * ns;
  const int rb = a.kq[Q * nk + kp];         // row block k' + Q of Theta for Omega'
  for (int n0 = 0; n0 < a.xq; n0 += npar) {
    for (int e = t; e < npar * NS * m; e += 256) {
      const int p = e / (NS * m), r = e - p * (NS * m);   // r = a m + l
      const int nn = n0 + p;
      ltb[e] = nn < a.xq ? a.Lt[((((long)Q * nk + k2) * a.xq + nn) * nkn + aoff) * m + r] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int n = n0 + nl;
    if (nl < npar && n < a.xq) {
      const double2* lt = ltb + (long)nl * NS * m;
      const double2* ltd = a.Ltd + ((((long)Q * nk + kp) * a.xq + n) * nkn + aoff + b) * m;
      double2 om[NS], omd[NS];
#pragma unroll
      for (int q = 0; q < NS; ++q) om[q] = omd[q] = make_double2(0.0, 0.0);
      for (int l = 0; l < m; ++l) {
        const double2 xa = thA[l * N + c];
        const double2 xd = ltd[l];
        const double2* tb = thB + (rb * m + l) * ns;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          om[q] = cadd(om[q], cmul(lt[q * m + l], xa));
          omd[q] = cadd(omd[q], cmul(xd, tb[q]));
        }
      }
      double2 ek = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < NS; ++q) ek = cadd(ek, cmul(om[q], omd[q]));
      double2 tl = make_double2(0.0, 0.0), tld = make_double2(0.0, 0.0);
      if (kp == k1) {
#pragma unroll
        for (int q = 0; q < NS; ++q)
          if (q == b) {
            tl = om[q];
            tld = omd[q];
          }
      }
      double2* o = pp + ((long)nl * N + c) * 3;
      o[0] = ek;
      o[1] = tl;
      o[2] = tld;
    }
    __syncthreads();
    if (t < npar * 3) {
      const int q = t / 3, j = t - q * 3, nn = n0 + q;
      if (nn < a.xq) {
        double2 v = make_double2(0.0, 0.0);
        for (int cc = 0; cc < N; ++cc) v = cadd(v, pp[((long)q * N + cc) * 3 + j]);
        wp[nn * 3 + j] = v;
      }
    }
    __syncthreads();
  }
  double2* out = a.part + ((((long)w * 2 + sp) * nk + Q) * a.xq) * nk * 3;
  for (int e = t; e < a.xq * 3; e += 256) {
    const int n = e / 3, j = e - n * 3;
    out[((long)n * nk + k1) * 3 + j] = wp[n * 3 + j];
  }
}

// ---------------------------------------------------------------------------
// the same traces on FP64 MFMA (v_mfma_f64_16x16x4f64, a complex product as
// four real ones). One workgroup per (group of G row blocks k1_j = G grp + j,
// walker, Q) and spin, G ns <= 16, Q the slowest grid index as in the VALU
// kernel. For each block of VB vectors, rows (n, a):
//   Omega'_{k'}[(n,b), (j,a)] = sum_l Ltd^{Q,k'}_n[b][l] Theta[(k'+Q, l), (k1_j, a)]
//     for every k', computed transposed (rows (j, a): one 16-row tile, the
//     staged Theta columns the A operand shared by KT column tiles (n, b) of
//     Ltd rows) and kept in LDS;
//   Omega_j[(n,a), c] = sum_l Lt^{Q,k2_j}_n[a][l] Theta[(k2_j, l), c]
//     (k2_j + Q = k1_j, c = (k', b) over the trial block), computed
//     transposed too (KT row tiles c of the staged Theta rows against one
//     column tile (n, a) of Lt rows), whose epilogue pairs every element with
//     Omega'_{k'}[(n,b), (j,a)].
// A unit is KT output tiles sharing one operand (2 KT independent accumulator
// chains), the contraction over l in KS steps of 4; the operand read from
// global memory (Ltd or Lt rows) goes straight into registers, the next
// unit's while this one multiplies. A lane's share of tr(Omega Omega') for its
// column (n, a) is summed over its rows and the unit's tiles in registers,
// then over the four row groups of the tile, the units and the rows of a
// vector in a fixed order (bitwise repeatable). The Omega' rows in LDS are an
// odd number of 16-byte slots apart, so a wave's accesses along (n, b) do not
// collide in the banks.
// ---------------------------------------------------------------------------
typedef __attribute__((ext_vector_type(4))) double kd4;
typedef __attribute__((ext_vector_type(2))) double kv2;         // (Re, Im)
typedef const __attribute__((address_space(1))) kv2 kp_g2;       // global memory
typedef __attribute__((address_space(3))) kv2 kp_l2;             // LDS
constexpr int KT = 3;             // output tiles per unit
constexpr int KP_MFMA_MAX_M = 32; // larger m: the unit's operand registers would spill
constexpr int KP_MFMA_MAX_NK = 64;

// dynamic LDS of the MFMA trace kernel: the Theta blocks G x 4KS x N and
// nk x 4KS x G ns (contraction rows padded with zeros to a multiple of 4), the
// Omega' of a vector block (VB vectors of nk ns rows GSP apart, one slot of
// padding per vector) and the row partials
static size_t kp_mfma_lds(int nk, int m, int ns, int G, int VB) {
  const size_t N = (size_t)nk * ns, GS = (size_t)G * ns, m4 = ((size_t)m + 3) / 4 * 4;
  const size_t r16 = ((size_t)VB * ns + 15) / 16 * 16, nch = ((N + 15) / 16 + KT - 1) / KT;
  return ((size_t)G * m4 * N + (size_t)nk * m4 * GS + (size_t)VB * (nk * ns * (GS | 1) + 1) +
          (size_t)G * (nch + 1) * r16) * 16;
}

// G: the largest divisor of nk with G ns <= 16; VB: the largest vector block
// that fits in LDS. False when the shape needs the VALU kernel.
static bool kp_mfma_shape(int nk, int m, int ns, int xq, int* G_out, int* VB_out, size_t* lds_out) {
  if (ns < 1 || ns > 16 || m > KP_MFMA_MAX_M || nk > KP_MFMA_MAX_NK) return false;
  int G = 1;
  for (int g = 1; g <= nk; ++g)
    if (nk % g == 0 && g * ns <= 16) G = g;
  int VB = 0;
  for (int v = 1; v <= xq; ++v)   // 1 KB left for the kernel's static tables
    if (kp_mfma_lds(nk, m, ns, G, v) + 1024 <= KP_MAX_LDS) VB = v;
  if (VB == 0) return false;
  *G_out = G;
  *VB_out = VB;
  *lds_out = kp_mfma_lds(nk, m, ns, G, VB);
  return true;
}

// x / d for 0 <= x < 2^22, rcp = 1 / d: (x + 1/2) / d lies at least 1 / (2 d)
// from an integer, and the float products err by less than (x + 1/2) 2^-23 / d
__device__ inline int kp_div(int x, float rcp) { return (int)(((float)x + 0.5f) * rcp); }

// KT complex tile products, one shared operand sh (A when SH_A, else B) and
// one per tile: the four real products of each tile are issued in four
// rounds over the tiles, so products into one accumulator are 2 KT - 1 apart;
// the shared operand's imaginary part is negated once
template <bool SH_A>
__device__ inline void kp_cmma_kt(kd4 (&cr)[KT], kd4 (&ci)[KT], kv2 sh, const kv2 (&v)[KT]) {
  const double nsy = -sh.y;
#pragma unroll
  for (int c = 0; c < KT; ++c)
    cr[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(SH_A ? sh.x : v[c].x, SH_A ? v[c].x : sh.x, cr[c], 0, 0, 0);
#pragma unroll
  for (int c = 0; c < KT; ++c)   // Re A Im B
    ci[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(SH_A ? sh.x : v[c].x, SH_A ? v[c].y : sh.y, ci[c], 0, 0, 0);
#pragma unroll
  for (int c = 0; c < KT; ++c)   // - Im A Im B
    cr[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(SH_A ? nsy : v[c].y, SH_A ? v[c].y : nsy, cr[c], 0, 0, 0);
#pragma unroll
  for (int c = 0; c < KT; ++c)   // Im A Re B
    ci[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(SH_A ? sh.y : v[c].y, SH_A ? v[c].x : sh.x, ci[c], 0, 0, 0);
}

// Lt / Ltd row (n, b) of the vector block at blk (row < R: (n0 + n) nkn + aoff
// + b after the block start), contraction elements 4 s + lq (clamped to m - 1:
// the staged Theta rows past m are zero)
template <int KS>
__device__ inline void kp_load_row(kp_g2* blk, int row, float rns, int ns, int nkn, int m, int lq, kv2 (&v)[KS]) {
  const int nl = kp_div(row, rns), b = row - nl * ns;
  kp_g2* p = blk + ((long)nl * nkn + b) * m;
#pragma unroll
  for (int s = 0; s < KS; ++s) v[s] = p[min(4 * s + lq, m - 1)];
}

// operands of a unit. Step 1 (Omega'^T), unit u = (k', chunk of KT column
// tiles): the KT Ltd row tiles of the vector block starting at n0 (R rows).
// Step 2 (Omega^T), unit u = (j, column tile, chunk): one Lt row tile of the
// block (Q, k2), whose (n, 0) rows start at blk2.
struct KpUnitGeo {
  int nk, xq, nkn, aoff, m, ns, nch1, nrt, nch2;
  float rns, rnch1, rnch2, rnrt2;
};
template <int KS>
__device__ inline void kp_load_u1(kp_g2* Ltd, int Q, const KpUnitGeo& g, int n0, int R, int u, int lr, int lq,
                                  kv2 (&v)[KT][KS]) {
  const int kp = kp_div(u, g.rnch1), ch = u - kp * g.nch1;
  kp_g2* blk = Ltd + ((((long)Q * g.nk + kp) * g.xq + n0) * g.nkn + g.aoff) * g.m;
#pragma unroll
  for (int c = 0; c < KT; ++c)
    kp_load_row<KS>(blk, min(16 * (KT * ch + c) + lr, R - 1), g.rns, g.ns, g.nkn, g.m, lq, v[c]);
}
template <int KS>
__device__ inline void kp_load_u2(kp_g2* Lt, int Q, int k2, const KpUnitGeo& g, int n0, int R, int u, int lr, int lq,
                                  kv2 (&v)[KS]) {
  const int j = kp_div(u, g.rnrt2), ct = kp_div(u - j * g.nrt * g.nch2, g.rnch2);
  kp_g2* blk = Lt + ((((long)Q * g.nk + k2) * g.xq + n0) * g.nkn + g.aoff) * g.m;
  kp_load_row<KS>(blk, min(16 * ct + lr, R - 1), g.rns, g.ns, g.nkn, g.m, lq, v);
}

// The LDS side of the kernel a unit needs
struct KpLdsGeo {
  kp_l2 *thA, *thB, *OP, *rp, *tp;
  long OPV;
  int M4, N, GS, GSP, R16, nch2, nrt, ns, grp, G;
  float rns, rnch2, rnrt2;
};

// step-1 unit u = (k', chunk ch of KT column tiles (n, b)): Omega'^T tiles
// into OP; rb = the Theta row block k' + Q
template <int KS>
__device__ inline void kp_unit1(const KpLdsGeo& L, const kv2 (&op)[KT][KS], int kp, int ch, int rb, int R, int lr,
                                int lq, int lrB) {
  kp_l2* bsrc = L.thB + (long)rb * L.M4 * L.GS + lrB;
  kd4 cr[KT], ci[KT];
#pragma unroll
  for (int c = 0; c < KT; ++c) cr[c] = ci[c] = kd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const kv2 av = bsrc[(4 * s + lq) * L.GS];
    kv2 bv[KT];
#pragma unroll
    for (int c = 0; c < KT; ++c) bv[c] = op[c][s];
    kp_cmma_kt<true>(cr, ci, av, bv);
  }
  // lane: column (n, b) = 16 ct + lr, rows (j, a) = lq + 4 i
#pragma unroll
  for (int c = 0; c < KT; ++c) {
    const int col = 16 * (KT * ch + c) + lr;
    if (col < R) {
      const int nl = kp_div(col, L.rns), b = col - nl * L.ns;
      kp_l2* o = L.OP + nl * L.OPV + ((long)kp * L.ns + b) * L.GSP;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (lq + 4 * i < L.GS) o[lq + 4 * i] = kv2{cr[c][i], ci[c][i]};
    }
  }
}

// step-2 unit u = (j, column tile ct (n, a), chunk ch of KT row tiles c):
// Omega^T tiles paired with Omega' (rp: the lane group's share of tr(Omega
// Omega'), tp: the diagonal of Omega_j)
template <int KS>
__device__ inline void kp_unit2(const KpLdsGeo& L, const kv2 (&op)[KS], int u, int R, int lr, int lq) {
  const int j = kp_div(u, L.rnrt2), rem = u - j * L.nrt * L.nch2, ct = kp_div(rem, L.rnch2), ch = rem - ct * L.nch2;
  const int k1 = L.grp * L.G + j, N = L.N, ns = L.ns;
  kp_l2* asrc = L.thA + (long)j * L.M4 * N;
  int arow[KT];
#pragma unroll
  for (int c = 0; c < KT; ++c) arow[c] = min(16 * (KT * ch + c) + lr, N - 1);   // rows c past N: dropped
  kd4 cr[KT], ci[KT];
#pragma unroll
  for (int c = 0; c < KT; ++c) cr[c] = ci[c] = kd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    kv2 av[KT];
#pragma unroll
    for (int c = 0; c < KT; ++c) av[c] = asrc[(long)(4 * s + lq) * N + arow[c]];
    kp_cmma_kt<false>(cr, ci, op[s], av);
  }
  // lane: column (n, a) = 16 ct + lr, rows c = 16 (KT ch + c) + lq + 4 i
  const int col = 16 * ct + lr, nl = kp_div(col, L.rns), aa = col - nl * ns;
  const bool cok = col < R;
  kp_l2* opn = L.OP + nl * L.OPV + j * ns + aa;
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int c = 0; c < KT; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rc = 16 * (KT * ch + c) + lq + 4 * i;
      if (cok && rc < N) {
        const int kpc = kp_div(rc, L.rns), bc = rc - kpc * ns;
        const kv2 o = opn[((long)kpc * ns + bc) * L.GSP];
        sr += cr[c][i] * o.x - ci[c][i] * o.y;
        si += cr[c][i] * o.y + ci[c][i] * o.x;
        if (kpc == k1 && bc == aa) L.tp[(long)j * L.R16 + col] = kv2{cr[c][i], ci[c][i]};
      }
    }
  sr += __shfl_xor(sr, 16);
  si += __shfl_xor(si, 16);
  sr += __shfl_xor(sr, 32);
  si += __shfl_xor(si, 32);
  if (lq == 0) L.rp[((long)j * L.nch2 + ch) * L.R16 + col] = kv2{sr, si};
}

template <int KS>
__global__ __launch_bounds__(256) void kp_trace_mfma_kernel(KpTraceArgs a, int sp, int G, int VB) {
  constexpr int M4 = 4 * KS;
  extern __shared__ kv2 lds_raw[];
  __shared__ int k2s[16], kqs[KP_MFMA_MAX_NK];
  const int grp = blockIdx.x, w = blockIdx.y, Q = blockIdx.z, t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6, lr = lane & 15, lq = lane >> 4;
  const int nk = a.nk, m = a.m, M = a.M, xq = a.xq;
  const int ns = sp ? a.nd : a.nu, N = nk * ns, GS = G * ns, GSP = GS | 1;
  const float rns = 1.0f / (float)ns;
  const int off = sp ? nk * a.nu : 0, aoff = sp ? a.nu : 0, nkn = a.nu + a.nd;
  const int R16 = (VB * ns + 15) / 16 * 16, nrt = R16 / 16, nct = (N + 15) / 16;
  const int nch1 = (nrt + KT - 1) / KT, nch2 = (nct + KT - 1) / KT;   // tile chunks
  const float rnch1 = 1.0f / (float)nch1, rnch2 = 1.0f / (float)nch2, rnrt2 = 1.0f / (float)(nrt * nch2);
  const long OPV = (long)nk * ns * GSP + 1;   // Omega' slots per vector
  kp_l2* thA = (kp_l2*)lds_raw;                 // [j][l < M4][c]: Theta[(k2_j, l), c], zero for l >= m
  kp_l2* thB = thA + (long)G * M4 * N;          // [k][l < M4][j ns + a]: Theta[(k, l), (k1_j, a)], zero for l >= m
  kp_l2* OP = thB + (long)nk * M4 * GS;         // [nl][k'][b][j ns + a]: Omega'_{k'}[(n0 + nl, b), (j, a)]
  kp_l2* rp = OP + (long)VB * OPV;              // [j][chunk][(n, a)]: shares of tr(Omega Omega')
  kp_l2* tp = rp + (long)G * nch2 * R16;        // [j][(n, a)]: the diagonal of Omega_j
  if (t < nk) kqs[t] = a.kq[Q * nk + t];        // the row block k' + Q
  __syncthreads();
  if (t < G) {
    const int k1 = grp * G + t;
    int k2 = 0;
    for (int c = 0; c < nk; ++c)
      if (kqs[c] == k1) k2 = c;
    k2s[t] = k2;
  }
  __syncthreads();
  kp_g2* th = (kp_g2*)a.thetaT + (long)w * a.ntot * M;
  for (int e = t; e < G * N * M4; e += 256) {   // l fastest: contiguous global reads
    const int j = e / (N * M4), r = e - j * N * M4, c = r / M4, l = r - c * M4;
    kv2 v = {0.0, 0.0};
    if (l < m) v = th[(long)(off + c) * M + k2s[j] * m + l];
    thA[((long)j * M4 + l) * N + c] = v;
  }
  for (int e = t; e < GS * nk * M4; e += 256) {
    const int ja = e / (nk * M4), r = e - ja * nk * M4, k = r / M4, l = r - k * M4, j = ja / ns, aa = ja - j * ns;
    kv2 v = {0.0, 0.0};
    if (l < m) v = th[(long)(off + (grp * G + j) * ns + aa) * M + k * m + l];
    thB[((long)k * M4 + l) * GS + ja] = v;
  }
  __syncthreads();
  double2* out = a.part + ((((long)w * 2 + sp) * nk + Q) * xq) * nk * 3;
  const int lrB = min(lr, GS - 1);   // A rows (j, a) past G ns: clamped reads, outputs dropped

  KpUnitGeo ug;
  ug.nk = nk; ug.xq = xq; ug.nkn = nkn; ug.aoff = aoff; ug.m = m; ug.ns = ns;
  ug.nch1 = nch1; ug.nrt = nrt; ug.nch2 = nch2;
  ug.rns = rns; ug.rnch1 = rnch1; ug.rnch2 = rnch2; ug.rnrt2 = rnrt2;
  KpLdsGeo L;
  L.thA = thA; L.thB = thB; L.OP = OP; L.rp = rp; L.tp = tp; L.OPV = OPV;
  L.M4 = M4; L.N = N; L.GS = GS; L.GSP = GSP; L.R16 = R16; L.nch2 = nch2; L.nrt = nrt; L.ns = ns;
  L.grp = grp; L.G = G; L.rns = rns; L.rnch2 = rnch2; L.rnrt2 = rnrt2;
  kp_g2* Ltd = (kp_g2*)a.Ltd;
  kp_g2* Lt = (kp_g2*)a.Lt;
  const int nu1 = nk * nch1, nu2 = G * nrt * nch2;
  // Operands come from global memory one unit ahead, in two register sets
  // used in turn (a copy between them would wait for the loads it copies).
  // Every unit issues the same loads, the last one of a wave re-reading its
  // own rows, so the wait before each multiply covers exactly the loads of
  // the unit it multiplies on every path.
  kv2 o1a[KT][KS], o1b[KT][KS], o2a[KS], o2b[KS];

  for (int n0 = 0; n0 < xq; n0 += VB) {
    const int vb = min(VB, xq - n0), R = vb * ns;
    // step 1: unit u in set A, u + 4 in set B, ...
    if (wave < nu1) kp_load_u1<KS>(Ltd, Q, ug, n0, R, wave, lr, lq, o1a);
    for (int u = wave; u < nu1; u += 8) {
      kp_load_u1<KS>(Ltd, Q, ug, n0, R, u + 4 < nu1 ? u + 4 : u, lr, lq, o1b);
      {
        const int kp = kp_div(u, rnch1);
        kp_unit1<KS>(L, o1a, kp, u - kp * nch1, kqs[kp], R, lr, lq, lrB);
      }
      if (u + 4 >= nu1) break;
      kp_load_u1<KS>(Ltd, Q, ug, n0, R, u + 8 < nu1 ? u + 8 : u + 4, lr, lq, o1a);
      const int kp = kp_div(u + 4, rnch1);
      kp_unit1<KS>(L, o1b, kp, u + 4 - kp * nch1, kqs[kp], R, lr, lq, lrB);
    }
    __syncthreads();
    // step 2: the same with the Omega units
    if (wave < nu2) kp_load_u2<KS>(Lt, Q, k2s[kp_div(wave, rnrt2)], ug, n0, R, wave, lr, lq, o2a);
    for (int u = wave; u < nu2; u += 8) {
      const int ub = u + 4 < nu2 ? u + 4 : u;
      kp_load_u2<KS>(Lt, Q, k2s[kp_div(ub, rnrt2)], ug, n0, R, ub, lr, lq, o2b);
      kp_unit2<KS>(L, o2a, u, R, lr, lq);
      if (u + 4 >= nu2) break;
      const int ua = u + 8 < nu2 ? u + 8 : u + 4;
      kp_load_u2<KS>(Lt, Q, k2s[kp_div(ua, rnrt2)], ug, n0, R, ua, lr, lq, o2a);
      kp_unit2<KS>(L, o2b, u + 4, R, lr, lq);
    }
    __syncthreads();
    // step 3: per (vector, j): tr(Omega Omega'), tr Omega, tr Omega'
    for (int e = t; e < vb * G; e += 256) {
      const int nl = e / G, j = e - nl * G, k1 = grp * G + j;
      kv2 ek = {0.0, 0.0}, tl = ek, tld = ek;
      for (int aa = 0; aa < ns; ++aa) {
        const int rr = nl * ns + aa;
        for (int ch = 0; ch < nch2; ++ch) ek += rp[((long)j * nch2 + ch) * R16 + rr];
        tl += tp[(long)j * R16 + rr];
        tld += OP[nl * OPV + ((long)k1 * ns + aa) * GSP + j * ns + aa];
      }
      double2* o = out + ((long)(n0 + nl) * nk + k1) * 3;
      o[0] = make_double2(ek.x, ek.y);
      o[1] = make_double2(tl.x, tl.y);
      o[2] = make_double2(tld.x, tld.y);
    }
    __syncthreads();
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

  KpTraceArgs a{};
  a.thetaT = w->theta.as<double2>();
  a.Lt = s->kp_Lt.as<double2>();
  a.Ltd = s->kp_Ltd.as<double2>();
  a.kq = s->kp_kq.as<int>();
  a.nk = nk; a.m = s->kp_m; a.xq = xq; a.nu = s->kp_nu; a.nd = s->kp_nd; a.ntot = s->ntot; a.M = s->M;
  a.part = w->kp_part.as<double2>();
  for (int sp = 0; sp < 2; ++sp) {
    const int ns = sp ? s->kp_nd : s->kp_nu;
    int G = 0, VB = 0;
    size_t lds = 0;
    // the MFMA kernel unless the walker set pins the VALU one (variant 1) or the shape needs it
    if (w->exch_var[sp] != 1 && kp_mfma_shape(nk, s->kp_m, ns, xq, &G, &VB, &lds)) {
      const int ks = ceil_div(s->kp_m, 4);
      switch (ks) {
#define AFQ_KP_KS(V)                                                                                          \
  case V:                                                                                                     \
    if (lds > 64 * 1024)                                                                                      \
      AFQ_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kp_trace_mfma_kernel<V>),                \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));                \
    hipLaunchKernelGGL(kp_trace_mfma_kernel<V>, dim3(nk / G, nw, nk), dim3(256), lds, st, a, sp, G, VB);     \
    break;
        AFQ_KP_KS(1) AFQ_KP_KS(2) AFQ_KP_KS(3) AFQ_KP_KS(4) AFQ_KP_KS(5) AFQ_KP_KS(6) AFQ_KP_KS(7) AFQ_KP_KS(8)
#undef AFQ_KP_KS
        default:
          AFQ_CHECK(false, AFQ_E_INVALID, "k-point trace kernel (MFMA): bad contraction length");
      }
      AFQ_TRY_HIP(hipGetLastError());
      continue;
    }
    switch (ns) {
#define AFQ_KP_NS(V)                                                                                   \
  case V:                                                                                              \
    if (s->kp_lds > 64 * 1024)                                                                         \
      AFQ_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kp_trace_kernel<V>),              \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)s->kp_lds));   \
    hipLaunchKernelGGL(kp_trace_kernel<V>, dim3(nk, nw, nk), dim3(256), s->kp_lds, st, a, sp);          \
    break;
      AFQ_KP_NS(1) AFQ_KP_NS(2) AFQ_KP_NS(3) AFQ_KP_NS(4) AFQ_KP_NS(5) AFQ_KP_NS(6) AFQ_KP_NS(7) AFQ_KP_NS(8)
      AFQ_KP_NS(9) AFQ_KP_NS(10) AFQ_KP_NS(11) AFQ_KP_NS(12) AFQ_KP_NS(13) AFQ_KP_NS(14) AFQ_KP_NS(15)
      AFQ_KP_NS(16)
#undef AFQ_KP_NS
      default:
        AFQ_CHECK(false, AFQ_E_UNSUPPORTED, "k-point trace kernel: at most 16 electrons per k-point and spin");
    }
    AFQ_TRY_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(kp_reduce_kernel, dim3(ceil_div(nk * xq, 256), 2 * nw), dim3(256), 0, st, w->kp_part.as<double2>(),
                     nk, xq, w->tro.as<double2>(), w->troo.as<double2>());
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
