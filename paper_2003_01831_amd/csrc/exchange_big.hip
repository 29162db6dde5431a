// Exchange/Coulomb contraction of the split-BF16x3 mode for 65..100 electrons
// per spin, tiled for one wave per SIMD:
//
//   * a workgroup is 4 waves covering two n-blocks of one walker; wave
//     (nb, part) computes the Re (part 0) or Im (part 1) plane of
//     Omega^{n0+nb}_w as a TM x TM tile of 16 x 16 MFMA tiles
//     (TM = ceil(N / 16)); rows and columns are stacked without per-block
//     padding in the packed operands;
//   * the waves share the walker operand (B) and the Cholesky operand (A)
//     through LDS. k advances in chunks of 32 through a three-stage ring of
//     LDS buffers filled by direct global->LDS loads (no register staging)
//     from wave-uniform addresses; the packed operands are chunk-major in HBM
//     (all rows of k-chunk 0, then chunk 1, ...), so the rows of one chunk
//     are one contiguous run. A chunk's fragments are held in registers and
//     refilled from the next chunk right after their last MFMA (the shared
//     split-BF16x3 chunk loop);
//   * fragments are read with 16-byte LDS loads from an XOR-swizzled layout;
//   * epilogue: every wave stores the lower triangle of its plane in LDS
//     (packed triangular layout) and reads the transposed partners of its
//     upper-triangle elements from its own and the other plane of the block,
//     giving tr Omega and tr(Omega Omega) without any HBM traffic;
//   * workgroups are ordered XCD by XCD in 2-D tiles of (n-pair, walker) so
//     the operands of resident workgroups are shared in each XCD's L2.
//
// Arithmetic: split-BF16x3 on v_mfma_f32_16x16x32_bf16 (hi*hi + hi*lo + lo*hi),
// FP32 accumulation.
#include <algorithm>
#include "common.h"
#include "mfma_ring.h"
#include "exchange_big.h"

namespace {

using ring::f4;
using ring::KC;
using ring::lds_t;
using ring::ROWB;

constexpr int NWAVE = 4;

constexpr int NMAX = 100;           // largest N

// Start (in floats) of row x of the padded lower-triangle layout used by the
// epilogue. Row y holds L(y) = 4 + 32 ceil((y - 3) / 32) floats (4 for y <= 3),
// at least y + 1, a multiple of 4 and congruent to 4 mod 32, so that
//   * every row starts 16-byte aligned (one 16-byte read fetches a lane's four
//     partners),
//   * row x starts at 4x mod 32 words: the 8 lanes of a 16-byte read (8
//     consecutive rows) hit 8 different 4-bank groups, and rows x and x + 4
//     (the two 16-lane halves of a 4-byte store) start 16 banks apart.
__host__ __device__ constexpr int trow(int x) {
  return x < 4 ? 4 * x
               : 4 * x + 32 * ((x - 4) + 16 * ((x - 4) >> 5) * (((x - 4) >> 5) - 1) + ((x - 4) >> 5) * ((x - 4) & 31));
}

template <int TM> struct Geo {
  // rows staged per operand region: both blocks (2N rows) rounded to 16; the
  // tile of the second block overhangs by at most 8 rows into the next region
  // or the stage's slack (those rows only feed discarded outputs)
  static constexpr int RR = 32 * TM < 208 ? 32 * TM : 208;
  static constexpr int RI = RR / 16;                   // 1 KB load instructions per region
  static constexpr int REG = RR * ROWB;                // bytes per region
  static constexpr int STAGE = 4 * REG + 512;          // A hi, A lo, B hi, B lo + slack
  static constexpr int NE = 16 * TM < NMAX ? 16 * TM : NMAX;
  static_assert(2 * trow(NE) * 4 <= STAGE, "epilogue planes must fit one stage");
};

// workgroups resident on one XCD form TB n-pairs x TW walkers tiles
constexpr int NXCD = 8, TB = 4, TW = 8;

// the wave-uniform base of load q of chunk ch: qb[q] (the load's first row
// in chunk 0) plus ch chunk strides of its operand (A: rows_a rows, B: rows_b)
template <int NQ> struct ExbLoader {
  const unsigned char* qb[NQ];
  long astride, bstride;
  bool is_a[NQ];
  __device__ const unsigned char* src(int q, int ch) const { return qb[q] + (long)ch * (is_a[q] ? astride : bstride); }
};

template <int TM>
__global__ __launch_bounds__(256, 1) void exchange_big_kernel(ExchBigArgs g) {
  using G = Geo<TM>;
  constexpr int RI = G::RI, REG = G::REG;
  __shared__ __align__(16) unsigned char L0[G::STAGE];
  __shared__ __align__(16) unsigned char L1[G::STAGE];
  __shared__ __align__(16) unsigned char L2[G::STAGE];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar address arithmetic
  const int N = g.n;
  const int nb = wave >> 1, part = wave & 1;      // n-block within the pair, plane
  // XCD-aware order: workgroup i runs on XCD i % 8; each XCD owns nw/8 walkers
  // and walks them in TB x TW tiles of (n-pair, walker) so that the tiles
  // resident at one time share their operands in that XCD's L2.
  int bn, w0;
  {
    const int pid = blockIdx.x;
    if (g.raster) {
      const int x = pid % NXCD, t = pid / NXCD;
      const int wpx = g.nw / NXCD, ntw = wpx / TW;
      const int tile = t / (TB * TW), r = t - tile * (TB * TW);
      bn = (tile / ntw) * TB + r / TW;
      w0 = x * wpx + (tile % ntw) * TW + r % TW;
    } else {
      bn = pid / g.nw;
      w0 = pid - bn * g.nw;
    }
  }
  const int n0 = 2 * bn;                          // first n-block of the workgroup
  const long arow0 = (long)n0 * N;
  const long brow0 = (long)w0 * 2 * N;

  // Load q of this wave (q < RI) moves 1 KB: instruction t = 4 q + wave of the
  // chunk, region t / RI (A hi, A lo, B hi, B lo), rows 16 (t % RI) ... + 15.
  ExbLoader<RI> ld;
  ld.astride = g.rows_a * (long)ROWB;
  ld.bstride = g.rows_b * (long)ROWB;
#pragma unroll
  for (int q = 0; q < RI; ++q) {
    const int t = q * NWAVE + wave, reg = t / RI, j = t - reg * RI;
    const unsigned char* base = static_cast<const unsigned char*>(reg == 0 ? g.a[0] : reg == 1 ? g.a[1]
                                                                   : reg == 2 ? g.b[0] : g.b[1]);
    ld.is_a[q] = reg < 2;
    ld.qb[q] = base + ((reg < 2 ? arow0 : brow0) + 16 * j) * ROWB;
  }
  __shared__ float trash[NWAVE * 64];             // the epilogue's sink for out-of-range elements
  f4 acc[TM][TM];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int arow = nb * N, brow = part * N;       // this wave's first rows in the A / B regions
  ring::bf3_stream<TM, TM, REG, REG, RI>(acc, (const lds_t*)L0, (const lds_t*)L1, (const lds_t*)L2, g.kp / KC, arow,
                                         brow, lane, wave, ld);
  __syncthreads();

  // ---- epilogue: lower triangles of both planes of each block in LDS ----
  // tr(Omega Omega) = sum_a Omega_aa^2 + 2 sum_{a<b} Omega_ab Omega_ba: waves
  // store the elements a >= b of their plane and read, for their elements
  // a <= b, the partners (b, a). Rows are padded (row x starts at trow(x)), so
  // the four partners (b, a..a+3) of a lane's four accumulator rows are one
  // aligned 16-byte read and neither stores nor reads conflict on banks. Branch-free:
  // out-of-range lanes store to a private trash slot and read a clamped
  // address; masked terms are selected to zero (the padding may hold anything).
  // Products of the FP32 accumulators are formed in FP64 (exact).
  float* pl = reinterpret_cast<float*>(nb == 0 ? L0 : L1);
  const int T4 = trow(N);
  float* mine = pl + part * T4;
  const float* other = pl + (part ^ 1) * T4;
  float* my_trash = trash + wave * 64 + lane;
  const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      const int b = 16 * j + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * i + 4 * lq + r;
        // tiles before the last row/column lie inside the block (16 (TM-1) < N)
        const bool ok = (i < TM - 1 || a < N) && (i > j || a >= b);
        float* dst = ok ? mine + (trow(a) + b) : my_trash;
        *dst = acc[i][j][r];
      }
    }
  __syncthreads();
  double s[5] = {0, 0, 0, 0, 0};   // tr_re, tr_im, rere, imim, reim
  double d_diag = 0.0, d_same = 0.0, d_other = 0.0;
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    const int b = 16 * j + lr;
    const bool okb = j < TM - 1 || b < N;
    const int tb = trow(b);
#pragma unroll
    for (int i = 0; i <= j; ++i) {
      const int a0 = 16 * i + 4 * lq;
      const int idx = okb ? tb + a0 : 0;
      const float4 pm = *reinterpret_cast<const float4*>(mine + idx);
      const float4 po = *reinterpret_cast<const float4*>(other + idx);
      const float pmv[4] = {pm.x, pm.y, pm.z, pm.w}, pov[4] = {po.x, po.y, po.z, po.w};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + r;
        const bool ok = okb && (i < j || a <= b);
        const double v = ok ? (double)acc[i][j][r] : 0.0;
        const double ps = ok ? (double)pmv[r] : 0.0, po_ = ok ? (double)pov[r] : 0.0;
        if (i < j) {                       // whole tile above the diagonal: a < b
          d_same += 2.0 * v * ps;
          d_other += v * po_;
        } else {
          const double ws = a < b ? 2.0 : 1.0;
          const double wo = (a < b || part == 0) ? 1.0 : 0.0;
          d_same += ws * v * ps;
          d_other += wo * v * po_;
          d_diag += a == b ? v : 0.0;
        }
      }
    }
  }
  s[part] = d_diag;
  s[2 + part] = d_same;
  s[4] = d_other;
#pragma unroll
  for (int q = 0; q < 5; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off);
  __shared__ double sums[NWAVE][5];
  if (lane == 0)
    for (int q = 0; q < 5; ++q) sums[wave][q] = s[q];
  __syncthreads();
  if (tid < 2) {
    const int nidx = n0 + tid;
    if (nidx < g.X) {
      double t[5];
      for (int q = 0; q < 5; ++q) t[q] = sums[2 * tid][q] + sums[2 * tid + 1][q];
      const long o = ((long)w0 * 2 + g.spin) * g.X + nidx;
      g.tro[o] = make_double2(t[0], t[1]);
      g.troo[o] = make_double2(t[2] - t[3], 2.0 * t[4]);
    }
  }
}

template <int TM>
int launch_tm(ExchBigArgs g, hipStream_t st) {
  AFQ_CHECK(g.n <= 16 * TM && g.n > 16 * (TM - 1), AFQ_E_INVALID, "exchange: tile does not cover the block");
  AFQ_CHECK(2 * g.n <= Geo<TM>::RR, AFQ_E_INVALID, "exchange: staged rows do not cover two blocks");
  AFQ_CHECK(g.kp % KC == 0 && g.kp >= 2 * KC, AFQ_E_INVALID, "exchange: contraction length must be a multiple of 32");
  // the last workgroup stages RR rows from its first row: they must lie in the arrays
  AFQ_CHECK((long)(g.X - 2 + g.X % 2) * g.n + Geo<TM>::RR <= g.rows_a &&
                (long)(g.nw - 1) * 2 * g.n + Geo<TM>::RR <= g.rows_b,
            AFQ_E_INVALID, "exchange: packed operands lack padding rows");
  const long nbn = ceil_div(g.X, 2);
  const long grid = nbn * g.nw;
  AFQ_CHECK(grid < (1l << 31), AFQ_E_INVALID, "exchange: grid too large");
  g.raster = (nbn % TB == 0) && (g.nw % (NXCD * TW) == 0);
  hipLaunchKernelGGL(exchange_big_kernel<TM>, dim3((unsigned)grid), dim3(256), 0, st, g);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

}  // namespace

bool exch_big_supported(int prec, int n) { return prec == AFQ_BF16X3 && n >= 65 && n <= NMAX; }

int exchange_big_launch(const ExchBigArgs& g, int prec, hipStream_t st) {
  AFQ_CHECK(exch_big_supported(prec, g.n), AFQ_E_INVALID, "exchange: needs split-BF16x3 and 65 <= N <= 100");
  switch ((g.n + 15) / 16) {
    case 5: return launch_tm<5>(g, st);
    case 6: return launch_tm<6>(g, st);
    default: return launch_tm<7>(g, st);
  }
}

int exch_big_kchunk() { return 2 * KC; }
int exch_big_kchunk_major() { return KC; }
