// System set-up: device copies of h1, L^n and the trial; the normal-ordering
// corrected one-body matrix h' = h - 1/2 sum_n L^n L^n; the half-rotated
// ht = T^H h and Lt^n = T^H L^n; the packed exchange operands per precision;
// and B1 = exp(-dt h'/2) by Taylor series with scaling and squaring.
#include <cmath>
#include "common.h"
#include "step_kernels.h"
#include "exchange_big.h"

int DevBuf::alloc(size_t n) {
  free();
  if (n == 0) return AFQ_OK;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    afq_set_error(std::string("hipMalloc(") + std::to_string(n) + " bytes): " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? AFQ_E_NOMEM : AFQ_E_HIP;
  }
  bytes = n;
  return AFQ_OK;
}

void DevBuf::free() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

static int real_gemm(int m, int n, int k, const double* A, long lda, int opA, const double* B, long ldb, int opB,
                     double* C, long ldc, double alpha, double beta, hipStream_t st) {
  GemmArgs<double> g = gemm_args<double>();
  g.m = m; g.n = n; g.k = k;
  g.A = A; g.lda = lda; g.opA = opA; g.cA = false;
  g.B = B; g.ldb = ldb; g.opB = opB; g.cB = false;
  g.C = C; g.ldc = ldc; g.cC = false;
  g.ar = alpha; g.br = beta;
  return gemm<double>(g, st);
}

int system_prepare_pack(afq_system s, int prec) {
  if (s->apack_prec == prec) return eri_sync(s);
  if (s->kp_nk > 0) {   // k-point systems have their own trace kernel and run in FP64
    AFQ_CHECK(prec == AFQ_FP64, AFQ_E_UNSUPPORTED, "k-point systems run in FP64 mode");
    s->apack_prec = s->prec = prec;
    return AFQ_OK;
  }
  if (s->apack_prec >= 0) ++s->version;
  const int kc = exch_kchunk(prec);
  const size_t esz = prec == AFQ_FP64 ? 8 : prec == AFQ_CFP32 ? 4 : 2;
  for (int sp = 0; sp < 2; ++sp) {
    PackShape& ps = s->ps[sp];
    ps.n = s->nspin_n(sp);
    ps.big = exch_big_supported(prec, ps.n);
    ps.np = ps.big ? ps.n : round_up(ps.n, 16);
    ps.pad = ps.big ? exch_big_pad_rows() : 0;
    ps.kcm = ps.big ? exch_big_kchunk_major() : 0;
    ps.ke = s->real_trial ? s->M : 2 * s->M;
    ps.kp = round_up(ps.ke, ps.big ? exch_big_kchunk() : kc);
    const size_t elems = ((size_t)s->X * ps.np + ps.pad) * ps.kp;
    AFQ_RET(s->apack[sp].alloc(elems * esz));
    if (prec == AFQ_BF16X3) AFQ_RET(s->apack_lo[sp].alloc(elems * esz));
    else s->apack_lo[sp].free();
    AFQ_RET(pack_a(prec, s->Lt.as<double2>(), s->X, s->ntot, s->M, s->spin_off(sp), ps, s->real_trial,
                   s->apack[sp].p, s->apack_lo[sp].p, s->stream));
  }
  if ((prec == AFQ_BF16X3 || prec == AFQ_FP64) && s->real_trial && !s->LtRe.p) {   // Coulomb GEMM and four-index set-up
    const long n = (long)s->X * s->ntot * s->M;
    AFQ_RET(s->LtRe.alloc(n * sizeof(double)));
    AFQ_RET(real_part(s->Lt.as<double2>(), s->LtRe.as<double>(), n, s->stream));
  }
  s->prec = prec;
  AFQ_RET(r32_prepare(s));
  AFQ_TRY_HIP(hipStreamSynchronize(s->stream));
  s->apack_prec = prec;
  s->eri_declined = false;
  return eri_sync(s);
}

// B1 = exp(Z), Z = -dt h'/2 (h' + sum_n c_n L^n with a background c): Z' =
// Z / 2^q with ||Z'||_inf <= 1/2, Horner evaluation of the order-18 Taylor
// polynomial, then q squarings.
int system_prepare_dt(afq_system s, double dt) {
  if (s->kp_nk > 0) return kp_prepare_dt(s, dt);
  if (s->B1.p && s->B1_dt == dt) return AFQ_OK;
  const int M = s->M;
  const size_t mm = (size_t)M * M;
  hipStream_t st = s->stream;
  if (!s->B1.p) AFQ_RET(s->B1.alloc(mm * sizeof(double)));
  DevBuf z, e0, e1, nrm;
  AFQ_RET(z.alloc(mm * sizeof(double)));
  AFQ_RET(e0.alloc(mm * sizeof(double)));
  AFQ_RET(e1.alloc(mm * sizeof(double)));
  AFQ_RET(nrm.alloc(sizeof(double)));
  const double* hsrc = s->mf_on ? s->hp_mf.as<double>() : s->hp.as<double>();
  AFQ_RET(launch_infnorm(hsrc, M, nrm.as<double>(), st));
  double hn = 0.0;
  AFQ_TRY_HIP(hipMemcpyAsync(&hn, nrm.p, sizeof(double), hipMemcpyDeviceToHost, st));
  AFQ_TRY_HIP(hipStreamSynchronize(st));
  const double zn = 0.5 * fabs(dt) * hn;
  int q = 0;
  while (zn / std::ldexp(1.0, q) > 0.5 && q < 60) ++q;
  const double scale = -0.5 * dt / std::ldexp(1.0, q);
  // z = h'; the factor `scale` is folded into each Horner step:
  // E_j = I + (scale / j) h' E_{j+1}, E_19 = I, E_1 = exp(scale h')
  AFQ_RET(copy_d(hsrc, z.as<double>(), (long)mm, st));
  const int order = 18;
  double* cur = e0.as<double>();
  double* nxt = e1.as<double>();
  AFQ_RET(fill_eye(cur, M, st));
  for (int j = order; j >= 1; --j) {
    AFQ_RET(fill_eye(nxt, M, st));
    AFQ_RET(real_gemm(M, M, M, z.as<double>(), M, OP_N, cur, M, OP_N, nxt, M, scale / j, 1.0, st));
    std::swap(cur, nxt);
  }
  for (int i = 0; i < q; ++i) {
    AFQ_RET(real_gemm(M, M, M, cur, M, OP_N, cur, M, OP_N, nxt, M, 1.0, 0.0, st));
    std::swap(cur, nxt);
  }
  AFQ_RET(copy_d(cur, s->B1.as<double>(), (long)mm, st));
  s->B1_dt = dt;
  AFQ_RET(r32_prepare_b1(s));
  AFQ_TRY_HIP(hipStreamSynchronize(st));
  return AFQ_OK;
}

int system_create_impl(afq_system* out, int M, int n_up, int n_dn, int X, const double* h1, const double* chol,
                       const double* phi_t, double e_core, int prec, void* stream, unsigned flags) {
  AFQ_CHECK(out, AFQ_E_INVALID, "afq_system_create: out is NULL");
  *out = nullptr;
  AFQ_CHECK(M >= 1 && M <= 4096, AFQ_E_INVALID, "afq_system_create: M must be in [1, 4096]");
  AFQ_CHECK(n_up >= 1 && n_dn >= 1 && n_up <= M && n_dn <= M, AFQ_E_INVALID,
            "afq_system_create: need 1 <= n_up, n_dn <= M");
  AFQ_CHECK(n_up <= 128 && n_dn <= 128, AFQ_E_UNSUPPORTED, "afq_system_create: at most 128 electrons per spin");
  AFQ_CHECK(X >= 1, AFQ_E_INVALID, "afq_system_create: n_chol must be >= 1");
  AFQ_CHECK(h1 && chol && phi_t, AFQ_E_INVALID, "afq_system_create: NULL input array");
  AFQ_CHECK(prec >= AFQ_FP64 && prec <= AFQ_BF16X3, AFQ_E_INVALID, "afq_system_create: unknown precision");
  AFQ_CHECK(std::isfinite(e_core), AFQ_E_INVALID, "afq_system_create: e_core is not finite");
  AFQ_CHECK((flags & ~AFQ_HOST_PTRS) == 0, AFQ_E_INVALID, "afq_system_create: unknown flag");
  const hipMemcpyKind in_kind = (flags & AFQ_HOST_PTRS) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  afq_system s = new afq_system_s();
  int rc = [&]() -> int {
    s->M = M; s->n_up = n_up; s->n_dn = n_dn; s->X = X; s->ntot = n_up + n_dn;
    s->e_core = e_core;
    s->stream = static_cast<hipStream_t>(stream);
    AFQ_TRY_HIP(hipGetDevice(&s->device));
    hipStream_t st = s->stream;
    const size_t mm = (size_t)M * M;
    AFQ_RET(s->h1.alloc(mm * 8));
    AFQ_RET(s->chol.alloc((size_t)X * mm * 8));
    AFQ_RET(s->phi.alloc((size_t)M * s->ntot * 16));
    // host inputs are pageable memory: the copies are complete once the
    // stream is synchronised below, before this call returns
    AFQ_TRY_HIP(hipMemcpyAsync(s->h1.p, h1, mm * 8, in_kind, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->chol.p, chol, (size_t)X * mm * 8, in_kind, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->phi.p, phi_t, (size_t)M * s->ntot * 16, in_kind, st));
    // validation: symmetry of h1 and every L^n, finiteness, real/complex trial
    DevBuf chk;
    AFQ_RET(chk.alloc(5 * sizeof(double)));
    AFQ_RET(fill_d(chk.as<double>(), 0.0, 5, st));
    AFQ_RET(launch_asym(s->h1.as<double>(), M, 1, chk.as<double>(), st));
    AFQ_RET(launch_asym(s->chol.as<double>(), M, X, chk.as<double>() + 2, st));
    AFQ_RET(launch_maximag(s->phi.as<double2>(), (long)M * s->ntot, chk.as<double>() + 4, st));
    double h[5];
    AFQ_TRY_HIP(hipMemcpyAsync(h, chk.p, sizeof(h), hipMemcpyDeviceToHost, st));
    AFQ_TRY_HIP(hipStreamSynchronize(st));
    AFQ_CHECK(std::isfinite(h[0]) && std::isfinite(h[1]) && std::isfinite(h[2]) && std::isfinite(h[3]),
              AFQ_E_INVALID, "afq_system_create: non-finite h1 or chol");
    AFQ_CHECK(h[0] <= 1e-12 * h[1] + 1e-300, AFQ_E_INVALID, "afq_system_create: h1 is not symmetric");
    AFQ_CHECK(h[2] <= 1e-12 * h[3] + 1e-300, AFQ_E_INVALID, "afq_system_create: a Cholesky vector is not symmetric");
    s->real_trial = h[4] == 0.0;
    if (s->real_trial) {
      AFQ_RET(s->phir.alloc((size_t)s->ntot * M * 8));
      AFQ_RET(real_part(s->phi.as<double2>(), s->phir.as<double>(), (long)M * s->ntot, st));
    }
    // h' = h - 1/2 sum_n L^n L^n = h - 1/2 Q^T Q with Q the (X M) x M stack of the symmetric L^n
    AFQ_RET(s->hp.alloc(mm * 8));
    AFQ_RET(copy_d(s->h1.as<double>(), s->hp.as<double>(), (long)mm, st));
    AFQ_RET(real_gemm(M, M, X * M, s->chol.as<double>(), M, OP_T, s->chol.as<double>(), M, OP_N,
                      s->hp.as<double>(), M, -0.5, 1.0, st));
    // ht = T^H h (ntot x M), Lt^n = T^H L^n (ntot x M each)
    AFQ_RET(s->ht.alloc((size_t)s->ntot * M * 16));
    AFQ_RET(s->Lt.alloc((size_t)X * s->ntot * M * 16));
    {
      GemmArgs<double> g = gemm_args<double>();
      g.m = s->ntot; g.n = M; g.k = M;
      g.A = s->phi.as<double>(); g.lda = s->ntot; g.opA = OP_C; g.cA = true;
      g.B = s->h1.as<double>(); g.ldb = M; g.cB = false;
      g.C = s->ht.as<double>(); g.ldc = M; g.cC = true;
      AFQ_RET(gemm<double>(g, st));
      g.B = s->chol.as<double>(); g.sB = (long)mm; g.batch = X;
      g.C = s->Lt.as<double>(); g.sC = (long)s->ntot * M;
      AFQ_RET(gemm<double>(g, st));
    }
    AFQ_RET(system_prepare_pack(s, prec));
    return AFQ_OK;
  }();
  if (rc != AFQ_OK) {
    delete s;
    return rc;
  }
  *out = s;
  return AFQ_OK;
}

// vmf[n] = Re sum_s tr(L^n T^s T^sH) = Re sum_{c,k} Lt[n][c][k] T[k][c], the
// trial's own force bias (one workgroup per vector, fixed-order tree)
__global__ __launch_bounds__(256) void mean_field_kernel(const double2* __restrict__ Lt,
                                                         const double2* __restrict__ phi, int ntot, int M,
                                                         double* __restrict__ vmf) {
  __shared__ double red[256];
  const int n = blockIdx.x, t = threadIdx.x;
  const long per = (long)ntot * M;
  const double2* l = Lt + (long)n * per;
  double acc = 0.0;
  for (long e = t; e < per; e += 256) {
    const long c = e / M, k = e - c * M;
    const double2 a = l[e], b = phi[k * ntot + c];
    acc += a.x * b.x - a.y * b.y;
  }
  red[t] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) vmf[n] = red[0];
}

// bad[0] = number of non-finite entries of x (one workgroup)
__global__ __launch_bounds__(256) void finite_count_kernel(const double* __restrict__ x, int n,
                                                           int* __restrict__ bad) {
  __shared__ int red[256];
  const int t = threadIdx.x;
  int c = 0;
  for (int i = t; i < n; i += 256) c += isfinite(x[i]) ? 0 : 1;
  red[t] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) bad[0] = red[0];
}

// Mean-field background subtraction: on = 0 switches it off; otherwise the
// background is the trial's own force bias (vmf_in NULL) or the caller's
// device vector of X doubles. Builds h' + sum_n c_n L^n and invalidates B1.
int system_set_background(afq_system s, int on, const double* vmf_in) {
  hipStream_t st = s->stream;
  const int M = s->M, X = s->X;
  const size_t mm = (size_t)M * M;
  if (!on) {
    if (!s->mf_on) return AFQ_OK;
    AFQ_TRY_HIP(hipStreamSynchronize(st));
    s->mf_on = false;
    s->vmf.free();
    s->hp_mf.free();
  } else {
    AFQ_RET(s->vmf.alloc((size_t)X * sizeof(double)));
    AFQ_RET(s->hp_mf.alloc(mm * sizeof(double)));
    if (vmf_in) {
      AFQ_TRY_HIP(hipMemcpyAsync(s->vmf.p, vmf_in, (size_t)X * sizeof(double), hipMemcpyDeviceToDevice, st));
      DevBuf bad;
      AFQ_RET(bad.alloc(sizeof(int)));
      hipLaunchKernelGGL(finite_count_kernel, dim3(1), dim3(256), 0, st, s->vmf.as<double>(), X, bad.as<int>());
      AFQ_TRY_HIP(hipGetLastError());
      int nbad = 0;
      AFQ_TRY_HIP(hipMemcpyAsync(&nbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
      AFQ_TRY_HIP(hipStreamSynchronize(st));
      if (nbad) {
        s->mf_on = false;
        s->vmf.free();
        s->hp_mf.free();
        AFQ_CHECK(false, AFQ_E_INVALID, "afq_system_set_background: the background vector is not finite");
      }
    } else {
      hipLaunchKernelGGL(mean_field_kernel, dim3(X), dim3(256), 0, st, s->Lt.as<double2>(), s->phi.as<double2>(),
                         s->ntot, M, s->vmf.as<double>());
      AFQ_TRY_HIP(hipGetLastError());
    }
    // h_mf = h' + sum_n c_n L^n : [1 x X] x [X x M^2]
    AFQ_RET(copy_d(s->hp.as<double>(), s->hp_mf.as<double>(), (long)mm, st));
    AFQ_RET(real_gemm(1, (int)mm, X, s->vmf.as<double>(), X, OP_N, s->chol.as<double>(), (long)mm, OP_N,
                      s->hp_mf.as<double>(), (long)mm, 1.0, 1.0, st));
    AFQ_TRY_HIP(hipStreamSynchronize(st));
    s->mf_on = true;
  }
  s->B1_dt = s->b1x_dt = s->b1x3_dt = -1.0;   // rebuilt by the next step's set-up
  ++s->b1_serial;
  ++s->version;
  return AFQ_OK;
}
