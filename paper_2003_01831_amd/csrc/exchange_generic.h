// Fused half-rotated Coulomb/exchange contraction (the dominant cost of the
// walker step; the dense 3-index "Energy" column of the paper's scaling table,
// O(x_c N^2 M^2) per walker):
//
//   Omega^{ns}_w = Lt^{ns} Theta^s_w          (N x N, never stored)
//   tro [w][s][n] = tr Omega^{ns}_w            (force bias / Coulomb)
//   troo[w][s][n] = tr(Omega^{ns}_w Omega^{ns}_w)   (exchange)
//
// As one GEMM per spin: C[(n,a)][(w,part,b)] = sum_k A[(n,a)][k] B[(w,part,b)][k]
// with A the packed half-rotated Cholesky rows and B the packed Theta^T rows
// (part 0 = Re, 1 = Im; a complex trial doubles k, see PackShape). Every
// workgroup owns PN whole n-blocks x PW whole walkers, so each N x N block and
// its transpose live in one workgroup: the traces are taken in the epilogue
// through LDS and Omega never reaches HBM.
//
// Arithmetic policies: FP64 MFMA (16x16x4 f64), FP32 MFMA (16x16x4 f32) and
// split-BF16x3 on BF16 MFMA (16x16x32 bf16: hi*hi + hi*lo + lo*hi, FP32
// accumulation). Each wave computes one n-block's rows (TM 16-row tiles) times
// DC 16-column tiles of one walker's [Re | Im] columns.
// Generic fused exchange kernel (template shared by the per-precision
// instantiation files exchange_f64.hip, exchange_f32.hip, exchange_bf16.hip).
#pragma once
#include <algorithm>
#include <type_traits>
#include "common.h"

namespace exch {


typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(4))) double d4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

struct PolF64 {
  using E = double;          // stored element
  using Acc = d4;
  using Frag = double;
  static constexpr int KSTEP = 4, KC = 16, PADE = 2, NPLANE = 1, ACC_REGS = 8;
  static constexpr int MUL = 1;
  // output row of (lane, r) inside a 16x16 tile
  __device__ static int orow(int lane, int r) { return (lane >> 4) + 4 * r; }
  __device__ static Frag frag(const E* base, int stride, int lane, int ks) {
    return base[(lane & 15) * stride + ks * KSTEP + (lane >> 4)];
  }
  __device__ static void mma(Acc& c, Frag a, Frag b) { c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

struct PolF32 {
  using E = float;
  using Acc = f4;
  using Frag = float;
  static constexpr int KSTEP = 4, KC = 32, PADE = 4, NPLANE = 1, ACC_REGS = 4;
  __device__ static int orow(int lane, int r) { return 4 * (lane >> 4) + r; }
  __device__ static Frag frag(const E* base, int stride, int lane, int ks) {
    return base[(lane & 15) * stride + ks * KSTEP + (lane >> 4)];
  }
  __device__ static void mma(Acc& c, Frag a, Frag b) { c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

struct PolBF16x3 {
  using E = unsigned short;  // bf16 bits
  using Acc = f4;
  using Frag = bf16x8;
  static constexpr int KSTEP = 32, KC = 32, PADE = 8, NPLANE = 2, ACC_REGS = 4;
  __device__ static int orow(int lane, int r) { return 4 * (lane >> 4) + r; }
  __device__ static Frag frag(const E* base, int stride, int lane, int ks) {
    const uint4 v = *reinterpret_cast<const uint4*>(base + (lane & 15) * stride + ks * KSTEP + 8 * (lane >> 4));
    return __builtin_bit_cast(Frag, v);
  }
  __device__ static void mma(Acc& c, Frag a, Frag b) { c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

template <class P> constexpr int dc_for(int tm, int budget) {
  int best = 1;
  for (int d = 1; d <= 2 * tm; ++d)
    if ((2 * tm) % d == 0 && tm * d * P::ACC_REGS <= budget) best = d;
  return best;
}

struct ExchArgs {
  const void* a_hi; const void* a_lo;   // packed A for this spin
  const void* b_hi; const void* b_lo;   // packed B for this spin
  int n, np, kp, X, nw, PN, PW, spin;
  int lds_kloop;                        // bytes of the k-loop staging
  int rb;                               // blocks per epilogue round
  double2* tro; double2* troo;          // [w][2][X]
};

// waves per workgroup: G waves per block times a power-of-two number of blocks
// (the PN x PW block grid below), at most about W waves in total
constexpr int pow2_floor(int x) { return x >= 2 ? 2 * pow2_floor(x / 2) : 1; }
template <int G, int W> constexpr int waves_total() { return G >= W ? G : G * pow2_floor(W / G); }

// Launch variants the autotuner chooses from: (target waves per workgroup,
// accumulator registers per wave). More waves stage more (n, walker) blocks
// per workgroup (more operand reuse per LDS byte); fewer waves leave more
// registers and LDS per block.
struct ExchVariant { int waves, budget; };
constexpr ExchVariant kExchVariants[] = {{8, 128}, {4, 128}, {16, 64}};
constexpr int kNumExchVariants = 3;

template <class P, int TM, int DC, int WV>
__global__ __launch_bounds__(64 * WV) void exchange_kernel(ExchArgs g) {
  using E = typename P::E;
  using Acc = typename P::Acc;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double partial[16][5];

  constexpr int G = 2 * TM / DC;        // waves per (n, w) block
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nthreads = blockDim.x;
  const int np = g.np, kp = g.kp;
  const int nblk_w = (g.nw + g.PW - 1) / g.PW;
  const int bn = blockIdx.x / nblk_w, bw = blockIdx.x - bn * nblk_w;
  const int n0 = bn * g.PN, w0 = bw * g.PW;
  const int bl = wave / G, gi = wave - bl * G;       // block-local index, column group
  const int nl = bl % g.PN, wl = bl / g.PN;

  const int stride = P::KC + P::PADE;                // LDS row stride (elements)
  const int rowsA = g.PN * np, rowsB = g.PW * 2 * np;
  E* lA = reinterpret_cast<E*>(smem);
  E* lB = lA + (size_t)rowsA * stride * P::NPLANE;

  Acc acc[TM][DC];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < DC; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  const long a_row0 = (long)n0 * np, a_rows_tot = (long)g.X * np;
  const long b_row0 = (long)w0 * 2 * np, b_rows_tot = (long)g.nw * 2 * np;
  constexpr int VPR = P::KC * (int)sizeof(E) / 16;   // 16-byte vectors per row chunk

  for (int k0 = 0; k0 < kp; k0 += P::KC) {
    __syncthreads();
    // stage A and B chunks (all planes) into LDS
    for (int pl = 0; pl < P::NPLANE; ++pl) {
      const E* ga = reinterpret_cast<const E*>(pl == 0 ? g.a_hi : g.a_lo);
      const E* gb = reinterpret_cast<const E*>(pl == 0 ? g.b_hi : g.b_lo);
      E* la = lA + (size_t)pl * rowsA * stride;
      E* lb = lB + (size_t)pl * rowsB * stride;
      for (int v = tid; v < rowsA * VPR; v += nthreads) {
        const int row = v / VPR, part = v - row * VPR;
        const long gr = a_row0 + row;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (gr < a_rows_tot)
          val = *reinterpret_cast<const uint4*>(ga + gr * kp + k0 + part * (16 / sizeof(E)));
        *reinterpret_cast<uint4*>(la + row * stride + part * (16 / sizeof(E))) = val;
      }
      for (int v = tid; v < rowsB * VPR; v += nthreads) {
        const int row = v / VPR, part = v - row * VPR;
        const long gr = b_row0 + row;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (gr < b_rows_tot)
          val = *reinterpret_cast<const uint4*>(gb + gr * kp + k0 + part * (16 / sizeof(E)));
        *reinterpret_cast<uint4*>(lb + row * stride + part * (16 / sizeof(E))) = val;
      }
    }
    __syncthreads();
    const E* wa = lA + (size_t)(nl * np) * stride;
    const E* wb = lB + (size_t)(wl * 2 * np + gi * DC * 16) * stride;
#pragma unroll
    for (int ks = 0; ks < P::KC / P::KSTEP; ++ks) {
      typename P::Frag af[TM], af_lo[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        af[i] = P::frag(wa + i * 16 * stride, stride, lane, ks);
        if constexpr (P::NPLANE == 2) af_lo[i] = P::frag(wa + (size_t)rowsA * stride + i * 16 * stride, stride, lane, ks);
      }
#pragma unroll
      for (int j = 0; j < DC; ++j) {
        const typename P::Frag bf = P::frag(wb + j * 16 * stride, stride, lane, ks);
        typename P::Frag bf_lo;
        if constexpr (P::NPLANE == 2) bf_lo = P::frag(wb + (size_t)rowsB * stride + j * 16 * stride, stride, lane, ks);
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          P::mma(acc[i][j], af[i], bf);
          if constexpr (P::NPLANE == 2) {
            P::mma(acc[i][j], af[i], bf_lo);
            P::mma(acc[i][j], af_lo[i], bf);
          }
        }
      }
    }
  }

  // ---------------- epilogue: traces through LDS ----------------
  // Each round stages rb whole blocks (Re and Im planes, n x n each) in LDS,
  // then the workgroup reduces tr Omega and tr Omega^2 of one block at a time
  // with a fixed-order reduction.
  using V = typename std::conditional<sizeof(E) == 8, double, float>::type;
  const int n = g.n, nn = n * n;
  V* tbuf = reinterpret_cast<V*>(smem);
  const int nblocks = g.PN * g.PW;
  const int nwaves = nthreads >> 6;
  for (int rb0 = 0; rb0 < nblocks; rb0 += g.rb) {
    const int rcount = min(g.rb, nblocks - rb0);
    __syncthreads();
    if (bl >= rb0 && bl < rb0 + rcount) {
      V* tb = tbuf + (size_t)(bl - rb0) * 2 * nn;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < DC; ++j) {
          const int cc = gi * DC * 16 + 16 * j + (lane & 15);
          const int part = cc >= 16 * TM;
          const int b = cc - part * 16 * TM;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int a = 16 * i + P::orow(lane, r);
            if (a < n && b < n) tb[part * nn + a * n + b] = (V)acc[i][j][r];
          }
        }
    }
    __syncthreads();
    for (int q = 0; q < rcount; ++q) {
      const V* tb = tbuf + (size_t)q * 2 * nn;
      double tr_re = 0, tr_im = 0, s_rere = 0, s_imim = 0, s_reim = 0;
      for (int e = tid; e < nn; e += nthreads) {
        const int a = e / n, b = e - a * n;
        const double rab = tb[e], iab = tb[nn + e];
        const double rba = tb[b * n + a], iba = tb[nn + b * n + a];
        s_rere += rab * rba;
        s_imim += iab * iba;
        s_reim += rab * iba;
        if (a == b) { tr_re += rab; tr_im += iab; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        tr_re += __shfl_xor(tr_re, off);
        tr_im += __shfl_xor(tr_im, off);
        s_rere += __shfl_xor(s_rere, off);
        s_imim += __shfl_xor(s_imim, off);
        s_reim += __shfl_xor(s_reim, off);
      }
      if (lane == 0) {
        partial[wave][0] = tr_re; partial[wave][1] = tr_im;
        partial[wave][2] = s_rere; partial[wave][3] = s_imim; partial[wave][4] = s_reim;
      }
      __syncthreads();
      if (tid == 0) {
        double sum[5] = {0, 0, 0, 0, 0};
        for (int v = 0; v < nwaves; ++v)
          for (int t = 0; t < 5; ++t) sum[t] += partial[v][t];
        const int blk = rb0 + q;
        const int nidx = n0 + blk % g.PN, widx = w0 + blk / g.PN;
        if (nidx < g.X && widx < g.nw) {
          const long o = ((long)widx * 2 + g.spin) * g.X + nidx;
          g.tro[o] = make_double2(sum[0], sum[1]);
          g.troo[o] = make_double2(sum[2] - sum[3], 2.0 * sum[4]);
        }
      }
      __syncthreads();
    }
  }
}

template <class P, int TM, int DC, int WV>
int launch_one(ExchArgs g, hipStream_t st) {
  constexpr int G = 2 * TM / DC;
  static_assert(WV <= 16, "too many waves per workgroup");
  // PN x PW blocks per workgroup with PN * PW = WV / G
  const int bpw = WV / G;
  int pn = 1, pw = 1;
  while (pn * pw < bpw) { if (pn <= pw) pn *= 2; else pw *= 2; }
  static_assert((WV / G) * G == WV && ((WV / G) & (WV / G - 1)) == 0, "blocks per workgroup must be a power of two");
  AFQ_CHECK(pn * pw == bpw, AFQ_E_INVALID, "exchange: block grid does not match the waves");
  g.PN = pn; g.PW = pw;
  const int waves = WV;
  const int stride = P::KC + P::PADE;
  const size_t kloop = (size_t)(pn * g.np + pw * 2 * g.np) * stride * sizeof(typename P::E) * P::NPLANE;
  using V = typename std::conditional<sizeof(typename P::E) == 8, double, float>::type;
  const size_t per_blk = 2 * (size_t)g.n * g.n * sizeof(V);   // Re and Im planes of one block
  const size_t budget = 160 * 1024 - 1024;
  AFQ_CHECK(per_blk <= budget, AFQ_E_UNSUPPORTED,
            "exchange: at most 100 electrons per spin in FP64 mode (the Omega block must fit in LDS)");
  int rb = (int)std::min<size_t>((size_t)pn * pw, std::max<size_t>(1, kloop / per_blk));
  if (rb < 1) rb = 1;
  size_t lds = std::max(kloop, rb * per_blk);
  AFQ_CHECK(lds <= budget, AFQ_E_UNSUPPORTED, "exchange: LDS requirement exceeds 159 KiB");
  g.rb = rb;
  g.lds_kloop = (int)kloop;
  const long nblk = (long)ceil_div(g.X, pn) * ceil_div(g.nw, pw);
  AFQ_CHECK(nblk < (1l << 31), AFQ_E_INVALID, "exchange: grid too large");
  hipLaunchKernelGGL((exchange_kernel<P, TM, DC, WV>), dim3((unsigned)nblk), dim3(64 * waves), lds, st, g);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}


template <class P, int TM, int V>
int launch_tv(ExchArgs g, hipStream_t st) {
  constexpr int DC = dc_for<P>(TM, kExchVariants[V].budget);
  constexpr int WV = waves_total<2 * TM / DC, kExchVariants[V].waves>();
  return launch_one<P, TM, DC, WV>(g, st);
}

template <class P, int TM>
int launch_t(ExchArgs g, int variant, hipStream_t st) {
  switch (variant) {
    case 0: return launch_tv<P, TM, 0>(g, st);
    case 1: return launch_tv<P, TM, 1>(g, st);
    case 2: return launch_tv<P, TM, 2>(g, st);
    default: break;
  }
  afq_set_error("exchange: unknown launch variant");
  return AFQ_E_INVALID;
}

template <class P>
int launch_policy(ExchArgs g, int variant, hipStream_t st) {
  switch (g.np / 16) {
    case 1: return launch_t<P, 1>(g, variant, st);
    case 2: return launch_t<P, 2>(g, variant, st);
    case 3: return launch_t<P, 3>(g, variant, st);
    case 4: return launch_t<P, 4>(g, variant, st);
    case 5: return launch_t<P, 5>(g, variant, st);
    case 6: return launch_t<P, 6>(g, variant, st);
    case 7: return launch_t<P, 7>(g, variant, st);
    case 8: return launch_t<P, 8>(g, variant, st);
    default: break;
  }
  afq_set_error("exchange: electrons per spin must be <= 128");
  return AFQ_E_UNSUPPORTED;
}

}  // namespace exch

// per-precision entry points (one translation unit each, compiled in parallel)
int exchange_generic_f64(const exch::ExchArgs& g, int variant, hipStream_t st);
int exchange_generic_f32(const exch::ExchArgs& g, int variant, hipStream_t st);
int exchange_generic_bf16(const exch::ExchArgs& g, int variant, hipStream_t st);
