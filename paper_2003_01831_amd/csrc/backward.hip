// Adjoint of the weighted mixed energy  f = scale * sum_w w_w Re E_L,w / sum_w w_w
// with the weights and the trial held fixed (E_L as in afq.h). With
// wh_w = scale * w_w / sum w, G = Theta T^H, Omega^n = Lt^n Theta and
// vbar_n = sum_s tr Omega^{ns}:
//
//   df/dh_ij   = Re sum_w wh_w sum_s G^s_ji            = Re (conj(T) Thbar^T)_ij
//   df/dL^n_ij = Re sum_w wh_w sum_s (vbar_n G - G L^n G)^s_ji
//              = Re sum_s (conj(T^s) Y^{ns T})_ij,
//                Y^{ns T} = sum_w wh_w (vbar_wn I - Omega^{ns}_w)^T Theta^{sT}_w
//   df/dW^s    = wh_w conj((I - G)^T Gamma S^-T),  grad = conj(Q) - T conj(Theta^T Q),
//                Q = Gamma S^-T,  Gamma^T = ht^s + sum_n (vbar_wn I - Omega^{ns}_w) Lt^{ns}
//
// Theta and Omega are recomputed (nothing is kept from the forward call);
// walkers are processed in chunks so the recomputed Omega blocks stay bounded.
// The three contractions of cost X N^2 M per walker-spin (Omega, Gamma, Y) run
// in the system's contraction precision (FP64, or FP32 in the reduced modes)
// with FP64 accumulation of Gamma and Y across chunks; the overlap inverse,
// Q, the gauge projection and the 1-RDM are FP64.
#include <algorithm>
#include "common.h"
#include "step_kernels.h"
#include "trace.h"

namespace {

int grid1(long n) { return (int)std::min<long>(std::max<long>(ceil_div(n, 256), 1), 65536); }

// wh_w = scale * w_w / sum_w w_w  (fixed-order reduction in one workgroup)
__global__ void wnorm_kernel(const double* __restrict__ w, int nw, double scale, double* __restrict__ wh) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nw; i += 256) s += w[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double tot = red[0];
  for (int i = threadIdx.x; i < nw; i += 256) wh[i] = tot > 0.0 ? scale * w[i] / tot : 0.0;
}

// thbar[c][k] = sum_w wh_w thetaT[w][c][k]  (fixed order over walkers)
__global__ void thbar_kernel(const double2* __restrict__ th, const double* __restrict__ wh, int nw, long per,
                             double2* __restrict__ out) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < per; e += (long)gridDim.x * blockDim.x) {
    double2 s = make_double2(0.0, 0.0);
    for (int w = 0; w < nw; ++w) s = cadd(s, cscale(th[(long)w * per + e], wh[w]));
    out[e] = s;
  }
}

// contiguous spin block in the contraction type: dst[r][k] = src[r * ld_r + k] (rows r of M elements)
template <typename T>
__global__ void gather_kernel(const double2* __restrict__ src, long nrows, int M, int rows_per_group, long grp_ld,
                              long row_ld, T* __restrict__ dst) {
  const long total = nrows * M;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long r = e / M;
    const int k = (int)(e - r * M);
    const long grp = r / rows_per_group, rr = r - grp * rows_per_group;
    const double2 v = src[grp * grp_ld + rr * row_ld + k];
    dst[2 * e] = (T)v.x;
    dst[2 * e + 1] = (T)v.y;
  }
}

// From Omega[w][n][a][b] of a walker chunk: Omega'' = vbar_wn delta_ab - Omega,
//   P [w][a][n][b] = Omega''             (rows a of the Gamma contraction, k = (n, b))
//   P2[n][b][w][a] = wh_w Omega''[w][n][a][b]   (rows b of the Y contraction, k = (w, a))
template <typename T>
__global__ void omega2_kernel(const T* __restrict__ om, const double2* __restrict__ tro, const double* __restrict__ wh,
                              int w0, int wc, int X, int N, T* __restrict__ P, T* __restrict__ P2) {
  const long nn = (long)N * N;
  const long total = (long)wc * X * nn;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int b = (int)(e % N);
    const long t = e / N;
    const int a = (int)(t % N);
    const long t2 = t / N;
    const int n = (int)(t2 % X);
    const int wl = (int)(t2 / X);
    const int w = w0 + wl;
    double vr = -(double)om[2 * e], vi = -(double)om[2 * e + 1];
    if (a == b) {
      const double2 vb = cadd(tro[((long)w * 2) * X + n], tro[((long)w * 2 + 1) * X + n]);
      vr += vb.x;
      vi += vb.y;
    }
    const long ip = (((long)wl * N + a) * X + n) * N + b;
    P[2 * ip] = (T)vr;
    P[2 * ip + 1] = (T)vi;
    const long ip2 = (((long)n * N + b) * wc + wl) * N + a;
    P2[2 * ip2] = (T)(wh[w] * vr);
    P2[2 * ip2 + 1] = (T)(wh[w] * vi);
  }
}

// Gamma^T_w := ht^s for every walker of the chunk
__global__ void gamma_init_kernel(const double2* __restrict__ ht, int off, int N, int M, int wc,
                                  double2* __restrict__ gam) {
  const long per = (long)N * M;
  const long total = per * wc;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
    gam[e] = ht[(long)off * M + e % per];
}

// grad[w][k][off + b] = wh_w (conj(Q[k][b]) - C2[k][b])
__global__ void dw_kernel(const double2* __restrict__ Q, const double2* __restrict__ C2, const double* __restrict__ wh,
                          int w0, int wc, int M, int N, int ntot, int off, double2* __restrict__ grad) {
  const long per = (long)M * N;
  const long total = per * wc;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int wl = (int)(e / per);
    const long r = e - wl * per;
    const int k = (int)(r / N), b = (int)(r - (long)k * N);
    const double2 q = Q[e], c = C2[e];
    const double s = wh[w0 + wl];
    grad[((long)(w0 + wl) * M + k) * ntot + off + b] = make_double2(s * (q.x - c.x), s * (-q.y - c.y));
  }
}

// out[b][i][j] = Re z[b][i][j]
__global__ void re_kernel(const double2* __restrict__ z, long n, double* __restrict__ out) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) out[e] = z[e].x;
}

template <typename T>
int backward_impl(afq_system s, afq_walkers w, double scale, double* d_h1, double* d_chol, double* d_walkers) {
  hipStream_t st = s->stream;
  const int M = s->M, ntot = s->ntot, X = s->X, nw = w->nw;
  const int nmax = std::max(s->n_up, s->n_dn);
  const long nm2 = (long)nmax * nmax;
  const long per = (long)M * ntot;
  // forward quantities at the current walkers: S^-1, Theta^T, vbar (tro)
  {
    AssembleArgs a{};
    a.dt = 0.0;
    AFQ_RET(compute_overlap_theta(s, w, w->W.as<double2>(), true, w->logdet.as<double2>()));
    AFQ_RET(pack_theta(s, w, st));
    AFQ_RET(exchange_launch(s, w, 0, st));
    AFQ_RET(exchange_launch(s, w, 1, st));
  }
  if (s->prec == AFQ_BF16X3) {
    // the backward contractions run in FP32; recompute tro in FP64 for vbar
    GemmArgs<double> g = gemm_args<double>();
    for (int sp = 0; sp < 2; ++sp) {
      const int n = s->nspin_n(sp), off = s->spin_off(sp);
      g.m = nw; g.n = X; g.k = n * M;
      g.A = w->theta.as<double>() + 2 * (long)off * M; g.lda = (long)ntot * M; g.cA = true;
      g.B = s->Lt.as<double>() + 2 * (long)off * M; g.ldb = (long)ntot * M; g.opB = OP_T; g.cB = true;
      g.C = w->tro.as<double>() + 2 * (long)sp * X; g.ldc = 2L * X; g.cC = true;
      AFQ_RET(gemm<double>(g, st));
    }
  }
  DevBuf wh;
  AFQ_RET(wh.alloc((size_t)nw * 8));
  hipLaunchKernelGGL(wnorm_kernel, dim3(1), dim3(256), 0, st, w->weights.as<double>(), nw, scale, wh.as<double>());
  AFQ_TRY_HIP(hipGetLastError());

  // d_h1 = Re sum_s conj(T^s) Thbar^{sT}
  if (d_h1) {
    DevBuf thb, tmp;
    AFQ_RET(thb.alloc((size_t)per * 16));
    AFQ_RET(tmp.alloc((size_t)M * M * 16));
    hipLaunchKernelGGL(thbar_kernel, dim3(grid1(per)), dim3(256), 0, st, w->theta.as<double2>(), wh.as<double>(), nw,
                       per, thb.as<double2>());
    AFQ_TRY_HIP(hipGetLastError());
    for (int sp = 0; sp < 2; ++sp) {
      const int n = s->nspin_n(sp), off = s->spin_off(sp);
      GemmArgs<double> g = gemm_args<double>();
      g.m = M; g.n = M; g.k = n;
      g.A = s->phi.as<double>() + 2 * off; g.lda = ntot; g.opA = OP_R; g.cA = true;
      g.B = thb.as<double>() + 2 * (long)off * M; g.ldb = M; g.cB = true;
      g.C = tmp.as<double>(); g.ldc = M; g.cC = true;
      g.br = sp == 0 ? 0.0 : 1.0;
      AFQ_RET(gemm<double>(g, st));
    }
    hipLaunchKernelGGL(re_kernel, dim3(grid1((long)M * M)), dim3(256), 0, st, tmp.as<double2>(), (long)M * M, d_h1);
    AFQ_TRY_HIP(hipGetLastError());
    AFQ_TRY_HIP(hipStreamSynchronize(st));   // tmp/thb are freed on return
  }
  if (!d_chol && !d_walkers) return AFQ_OK;

  // walker chunk so that the recomputed Omega and its two permuted copies fit in ~3 GiB
  const long blk = (long)X * nmax * nmax * 2 * sizeof(T);
  const int wc = (int)std::max<long>(1, std::min<long>(nw, (1l << 30) / std::max<long>(blk, 1)));
  DevBuf om, P, P2, lts, ths, gam, Q, R, C2, Y, cchol;
  AFQ_RET(om.alloc((size_t)wc * blk));
  AFQ_RET(P.alloc((size_t)wc * blk));
  AFQ_RET(P2.alloc((size_t)wc * blk));
  AFQ_RET(lts.alloc((size_t)X * nmax * M * 2 * sizeof(T)));
  AFQ_RET(ths.alloc((size_t)wc * nmax * M * 2 * sizeof(T)));
  if (d_walkers) {
    AFQ_RET(gam.alloc((size_t)wc * nmax * M * 16));
    AFQ_RET(Q.alloc((size_t)wc * M * nmax * 16));
    AFQ_RET(R.alloc((size_t)wc * nm2 * 16));
    AFQ_RET(C2.alloc((size_t)wc * M * nmax * 16));
  }
  if (d_chol) {
    AFQ_RET(Y.alloc((size_t)X * nmax * M * 16));
    AFQ_RET(cchol.alloc((size_t)X * M * M * 16));
  }
  for (int sp = 0; sp < 2; ++sp) {
    const int N = s->nspin_n(sp), off = s->spin_off(sp);
    // Lt^{s} rows (n, b) contiguous, in the contraction type
    hipLaunchKernelGGL(gather_kernel<T>, dim3(grid1((long)X * N * M)), dim3(256), 0, st, s->Lt.as<double2>(),
                       (long)X * N, M, N, (long)ntot * M, (long)M, lts.as<T>());
    AFQ_TRY_HIP(hipGetLastError());
    if (d_chol) AFQ_TRY_HIP(hipMemsetAsync(Y.p, 0, (size_t)X * N * M * 16, st));
    for (int w0 = 0; w0 < nw; w0 += wc) {
      const int cw = std::min(wc, nw - w0);
      // Theta^{sT} of the chunk, contiguous: ths[w][b][k]
      hipLaunchKernelGGL(gather_kernel<T>, dim3(grid1((long)cw * N * M)), dim3(256), 0, st,
                         w->theta.as<double2>() + ((long)w0 * ntot + off) * M, (long)cw * N, M, N, per, (long)M,
                         ths.as<T>());
      AFQ_TRY_HIP(hipGetLastError());
      // Omega[w][(n, a)][b] = Lt (X N x M) Theta_w (M x N)
      {
        GemmArgs<T> g = gemm_args<T>();
        g.m = X * N; g.n = N; g.k = M; g.batch = cw;
        g.A = lts.as<T>(); g.lda = M; g.cA = true; g.sA = 0;
        g.B = ths.as<T>(); g.ldb = M; g.opB = OP_T; g.cB = true; g.sB = (long)N * M;
        g.C = om.as<T>(); g.ldc = N; g.cC = true; g.sC = (long)X * N * N;
        AFQ_RET(gemm<T>(g, st));
      }
      hipLaunchKernelGGL(omega2_kernel<T>, dim3(grid1((long)cw * X * N * N)), dim3(256), 0, st, om.as<T>(),
                         w->tro.as<double2>(), wh.as<double>(), w0, cw, X, N, P.as<T>(), P2.as<T>());
      AFQ_TRY_HIP(hipGetLastError());
      if (d_chol) {
        // Y^{nT}[b][k] += sum_{(w, a)} P2[n][b][(w, a)] ths[(w, a)][k]
        GemmArgs<T> g = gemm_args<T>();
        g.m = N; g.n = M; g.k = cw * N; g.batch = X;
        g.A = P2.as<T>(); g.lda = (long)cw * N; g.cA = true; g.sA = (long)N * cw * N;
        g.B = ths.as<T>(); g.ldb = M; g.cB = true; g.sB = 0;
        g.D = Y.as<double2>(); g.ldd = M; g.sD = (long)N * M;
        AFQ_RET(gemm<T>(g, st));
      }
      if (d_walkers) {
        // Gamma^T_w = ht^s + P[w] (N x X N) Lt (X N x M)
        hipLaunchKernelGGL(gamma_init_kernel, dim3(grid1((long)cw * N * M)), dim3(256), 0, st,
                           s->ht.as<double2>(), off, N, M, cw, gam.as<double2>());
        AFQ_TRY_HIP(hipGetLastError());
        {
          GemmArgs<T> g = gemm_args<T>();
          g.m = N; g.n = M; g.k = X * N; g.batch = cw;
          g.A = P.as<T>(); g.lda = (long)X * N; g.cA = true; g.sA = (long)N * X * N;
          g.B = lts.as<T>(); g.ldb = M; g.cB = true; g.sB = 0;
          g.D = gam.as<double2>(); g.ldd = M; g.sD = (long)N * M;
          AFQ_RET(gemm<T>(g, st));
        }
        // Q = Gamma S^-T (M x N)
        GemmArgs<double> q = gemm_args<double>();
        q.m = M; q.n = N; q.k = N; q.batch = cw;
        q.A = gam.as<double>(); q.lda = M; q.opA = OP_T; q.cA = true; q.sA = (long)N * M;
        q.B = w->Sinv.as<double>() + 2 * ((long)w0 * 2 * nm2 + sp * nm2); q.ldb = N; q.opB = OP_T; q.cB = true;
        q.sB = 2 * nm2;
        q.C = Q.as<double>(); q.ldc = N; q.cC = true; q.sC = (long)M * N;
        AFQ_RET(gemm<double>(q, st));
        // R = Theta^T Q (N x N)
        GemmArgs<double> r = gemm_args<double>();
        r.m = N; r.n = N; r.k = M; r.batch = cw;
        r.A = w->theta.as<double>() + 2 * ((long)w0 * per + (long)off * M); r.lda = M; r.cA = true; r.sA = per;
        r.B = Q.as<double>(); r.ldb = N; r.cB = true; r.sB = (long)M * N;
        r.C = R.as<double>(); r.ldc = N; r.cC = true; r.sC = nm2;
        AFQ_RET(gemm<double>(r, st));
        // C2 = T conj(R) (M x N)
        GemmArgs<double> c = gemm_args<double>();
        c.m = M; c.n = N; c.k = N; c.batch = cw;
        c.A = s->phi.as<double>() + 2 * off; c.lda = ntot; c.cA = true; c.sA = 0;
        c.B = R.as<double>(); c.ldb = N; c.opB = OP_R; c.cB = true; c.sB = nm2;
        c.C = C2.as<double>(); c.ldc = N; c.cC = true; c.sC = (long)M * N;
        AFQ_RET(gemm<double>(c, st));
        hipLaunchKernelGGL(dw_kernel, dim3(grid1((long)cw * M * N)), dim3(256), 0, st, Q.as<double2>(),
                           C2.as<double2>(), wh.as<double>(), w0, cw, M, N, ntot, off,
                           reinterpret_cast<double2*>(d_walkers));
        AFQ_TRY_HIP(hipGetLastError());
      }
    }
    if (d_chol) {
      // d_chol[n] (+)= Re conj(T^s) Y^{nT}
      GemmArgs<double> g = gemm_args<double>();
      g.m = M; g.n = M; g.k = N; g.batch = X;
      g.A = s->phi.as<double>() + 2 * off; g.lda = ntot; g.opA = OP_R; g.cA = true; g.sA = 0;
      g.B = Y.as<double>(); g.ldb = M; g.cB = true; g.sB = (long)N * M;
      g.C = cchol.as<double>(); g.ldc = M; g.cC = true; g.sC = (long)M * M;
      g.br = sp == 0 ? 0.0 : 1.0;
      AFQ_RET(gemm<double>(g, st));
    }
  }
  if (d_chol) {
    hipLaunchKernelGGL(re_kernel, dim3(grid1((long)X * M * M)), dim3(256), 0, st, cchol.as<double2>(),
                       (long)X * M * M, d_chol);
    AFQ_TRY_HIP(hipGetLastError());
  }
  AFQ_TRY_HIP(hipStreamSynchronize(st));   // scratch buffers are freed on return
  return AFQ_OK;
}

}  // namespace

int energy_backward(afq_system s, afq_walkers w, double scale, double* d_h1, double* d_chol, double* d_walkers) {
  AFQ_RET(system_prepare_pack(s, s->prec));
  AFQ_RET(walkers_alloc_scratch(w));
  AFQ_CHECK(w->nw <= 65535, AFQ_E_INVALID, "afq_energy_backward: too many walkers");
  if (s->prec == AFQ_FP64) return backward_impl<double>(s, w, scale, d_h1, d_chol, d_walkers);
  return backward_impl<float>(s, w, scale, d_h1, d_chol, d_walkers);
}
