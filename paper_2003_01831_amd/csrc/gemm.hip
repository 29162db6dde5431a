// Generic batched complex GEMM for the small and medium contractions of the
// walker step (overlaps T^H W, Theta = W S^-1, B1 W, the Taylor products A V,
// the Gram matrices of QR, the A = sum_n c_n L^n build and the system set-up).
// 64 x 64 output tile per 256-thread workgroup, 4 x 4 complex outputs per
// thread, k staged through LDS in chunks of 16 as separate Re/Im planes.
#include "common.h"

namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 1;

template <typename T>
__device__ inline void load_elem(const T* p, long idx, bool cplx, bool conj, T& re, T& im) {
  if (cplx) {
    re = p[2 * idx];
    im = conj ? -p[2 * idx + 1] : p[2 * idx + 1];
  } else {
    re = p[idx];
    im = T(0);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs<T> g) {
  __shared__ T As_r[BK][BM + PAD], As_i[BK][BM + PAD];
  __shared__ T Bs_r[BK][BN + PAD], Bs_i[BK][BN + PAD];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const long b = blockIdx.z;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int es_a = g.cA ? 2 : 1, es_b = g.cB ? 2 : 1;
  const T* A = g.A + b * g.sA * es_a;
  const T* B = g.B + b * g.sB * es_b;
  const bool ca = g.opA == OP_C, cb = g.opB == OP_C;

  T acc_r[4][4], acc_i[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc_r[i][j] = acc_i[i][j] = T(0);

  for (int k0 = 0; k0 < g.k; k0 += BK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int kk, mm;
      if (g.opA == OP_N) { kk = e & 15; mm = e >> 4; } else { kk = e >> 6; mm = e & 63; }
      const int gi = m0 + mm, gk = k0 + kk;
      T re = T(0), im = T(0);
      if (gi < g.m && gk < g.k) {
        const long idx = g.opA == OP_N ? (long)gi * g.lda + gk : (long)gk * g.lda + gi;
        load_elem(A, idx, g.cA, ca, re, im);
      }
      As_r[kk][mm] = re;
      As_i[kk][mm] = im;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int kk, nn;
      if (g.opB == OP_N) { kk = e >> 6; nn = e & 63; } else { kk = e & 15; nn = e >> 4; }
      const int gj = n0 + nn, gk = k0 + kk;
      T re = T(0), im = T(0);
      if (gj < g.n && gk < g.k) {
        const long idx = g.opB == OP_N ? (long)gk * g.ldb + gj : (long)gj * g.ldb + gk;
        load_elem(B, idx, g.cB, cb, re, im);
      }
      Bs_r[kk][nn] = re;
      Bs_i[kk][nn] = im;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < BK; ++kk) {
      T ar[4], ai[4], br[4], bi[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) { ar[i] = As_r[kk][ty + 16 * i]; ai[i] = As_i[kk][ty + 16 * i]; }
#pragma unroll
      for (int j = 0; j < 4; ++j) { br[j] = Bs_r[kk][tx + 16 * j]; bi[j] = Bs_i[kk][tx + 16 * j]; }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc_r[i][j] += ar[i] * br[j] - ai[i] * bi[j];
          acc_i[i][j] += ar[i] * bi[j] + ai[i] * br[j];
        }
    }
    __syncthreads();
  }

  T* C = g.C ? g.C + b * g.sC * (g.cC ? 2 : 1) : nullptr;
  double2* D = g.D ? g.D + b * g.sD : nullptr;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gi = m0 + ty + 16 * i;
    if (gi >= g.m) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gj = n0 + tx + 16 * j;
      if (gj >= g.n) continue;
      double vr = g.ar * (double)acc_r[i][j] - g.ai * (double)acc_i[i][j];
      double vi = g.ar * (double)acc_i[i][j] + g.ai * (double)acc_r[i][j];
      if (C) {
        const long ci = (long)gi * g.ldc + gj;
        if (g.br != 0.0 || g.bi != 0.0) {
          double cr, cim;
          if (g.cC) { cr = C[2 * ci]; cim = C[2 * ci + 1]; } else { cr = C[ci]; cim = 0.0; }
          vr += g.br * cr - g.bi * cim;
          vi += g.br * cim + g.bi * cr;
        }
        if (g.cC) { C[2 * ci] = (T)vr; C[2 * ci + 1] = (T)vi; } else { C[ci] = (T)vr; }
      }
      if (D) {
        double2* d = D + (long)gi * g.ldd + gj;
        d->x += vr;
        d->y += vi;
      }
    }
  }
}

}  // namespace

template <typename T> GemmArgs<T> gemm_args() {
  GemmArgs<T> g{};
  g.batch = 1;
  g.ar = 1.0;
  g.opA = g.opB = OP_N;
  return g;
}

template <typename T> int gemm(const GemmArgs<T>& g, hipStream_t st) {
  AFQ_CHECK(g.m >= 0 && g.n >= 0 && g.k >= 0 && g.batch >= 0, AFQ_E_INVALID, "gemm: negative size");
  if (g.m == 0 || g.n == 0 || g.batch == 0) return AFQ_OK;
  AFQ_CHECK(g.A && g.B && (g.C || g.D), AFQ_E_INVALID, "gemm: null operand");
  AFQ_CHECK(g.batch <= 65535, AFQ_E_INVALID, "gemm: batch too large");
  dim3 grid(ceil_div(g.n, BN), ceil_div(g.m, BM), g.batch);
  AFQ_CHECK(grid.y <= 65535, AFQ_E_INVALID, "gemm: m too large");
  hipLaunchKernelGGL(gemm_kernel<T>, grid, dim3(256), 0, st, g);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

template int gemm<double>(const GemmArgs<double>&, hipStream_t);
template int gemm<float>(const GemmArgs<float>&, hipStream_t);
template GemmArgs<double> gemm_args<double>();
template GemmArgs<float> gemm_args<float>();
