// Exchange/Coulomb contraction of the split-BF16x3 mode for 65..100 electrons
// per spin, tiled for one wave per SIMD:
//
//   * a workgroup is 4 waves covering two n-blocks of one walker; wave
//     (nb, part) computes the Re (part 0) or Im (part 1) plane of
//     Omega^{n0+nb}_w as a TM x TM tile of 16 x 16 MFMA tiles
//     (TM = ceil(N / 16)); rows and columns are stacked without per-block
//     padding in the packed operands;
//   * the waves share the walker operand (B) and the Cholesky operand (A)
//     through LDS; k advances in chunks of 32 that are double-buffered with
//     direct global->LDS loads (no register staging), so the next chunk
//     streams in while the current one feeds the MFMAs; the two buffers are
//     distinct LDS objects so the compiler can tell the one being read from
//     the one being filled;
//   * fragments are read with 16-byte LDS loads from an XOR-swizzled layout;
//   * epilogue: every wave stores the lower-triangle tiles of its plane in LDS
//     (row stride N + 1, so the transposed reads are bank-conflict free) and
//     reads the transposed partners of its upper-triangle tiles from its own
//     and the other plane of the block, giving tr Omega and tr(Omega Omega)
//     without any HBM traffic;
//   * workgroups are ordered XCD by XCD in 2-D tiles of (n-pair, walker) so
//     the operands of resident workgroups are shared in each XCD's L2.
//
// Arithmetic: split-BF16x3 on v_mfma_f32_16x16x32_bf16 (hi*hi + hi*lo + lo*hi),
// FP32 accumulation, in two passes per chunk (hi*hi + hi*lo with the A hi
// fragments resident, then lo*hi with the A lo fragments resident).
#include <algorithm>
#include "common.h"
#include "exchange_big.h"

namespace {

typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((address_space(3))) unsigned char lds_t;

constexpr int KC = 32;              // k per chunk (bf16 elements); chunks come in pairs
constexpr int NWAVE = 4;
constexpr int ROWB = KC * 2;        // bytes per LDS row per plane
constexpr int CPR = ROWB / 16;      // 16-byte chunks per row

// XOR swizzle of the 16-byte chunks of a 64-byte row (an involution)
__device__ inline int swz(int row, int c) { return c ^ ((row >> 1) & 3); }

__device__ inline uint4 lds16(const unsigned char* p) { return *reinterpret_cast<const uint4*>(p); }

__device__ inline bf16x8 frag(const unsigned char* plane, int row, int lq) {
  return __builtin_bit_cast(bf16x8, lds16(plane + row * ROWB + 16 * swz(row, lq)));
}

constexpr int NMAX = 100;           // largest N: both planes of two blocks fit in LDS at once

template <int TM> struct Geo {
  static constexpr int ROWS = 32 * TM;                 // rows per operand region (>= N + 16 TM)
  static constexpr int BUF = 2 * ROWS * ROWB * 2;      // A and B, hi and lo
  static constexpr int NE = 16 * TM < NMAX ? 16 * TM : NMAX;
  static constexpr int EPI = 2 * NE * (NE + 1) * 4;    // Re and Im planes of one block, row stride N + 1
  static constexpr int SIZE = BUF > EPI ? BUF : EPI;   // bytes of each of the two LDS objects
};

// workgroups resident on one XCD form TB n-pairs x TW walkers tiles
constexpr int NXCD = 8, TB = 4, TW = 8;

// One chunk (32 k) of this wave's TM x TM tile. A planes at la (hi, then lo
// after ROWS rows), B planes at lb likewise.
template <int TM>
__device__ inline void mma_chunk(f4 (&acc)[TM][TM], const unsigned char* la, const unsigned char* lb, int arow,
                                 int brow, int lane) {
  constexpr int R = Geo<TM>::ROWS;
  const int lr = lane & 15, lq = lane >> 4;
  bf16x8 a[TM];
#pragma unroll
  for (int i = 0; i < TM; ++i) a[i] = frag(la, arow + 16 * i + lr, lq);
  bf16x8 bh = frag(lb, brow + lr, lq), bl = frag(lb + R * ROWB, brow + lr, lq);
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    bf16x8 nh = bh, nl = bl;
    if (j + 1 < TM) {
      nh = frag(lb, brow + 16 * (j + 1) + lr, lq);
      nl = frag(lb + R * ROWB, brow + 16 * (j + 1) + lr, lq);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bh, acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bl, acc[i][j], 0, 0, 0);
    }
    bh = nh;
    bl = nl;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) a[i] = frag(la + R * ROWB, arow + 16 * i + lr, lq);
  bh = frag(lb, brow + lr, lq);
#pragma unroll
  for (int j = 0; j < TM; ++j) {
    bf16x8 nh = bh;
    if (j + 1 < TM) nh = frag(lb, brow + 16 * (j + 1) + lr, lq);
#pragma unroll
    for (int i = 0; i < TM; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bh, acc[i][j], 0, 0, 0);
    bh = nh;
  }
}

// Direct global->LDS loads of one chunk of a region of `rows` rows of one
// plane: slot s of wave-instruction j holds row s/CPR, swizzled chunk s%CPR.
__device__ inline void dma_region(const unsigned char* g, long row0, long kp_bytes, long k0_bytes, lds_t* l,
                                  int rows, int wave, int lane) {
  const int ninstr = rows * ROWB / 1024;
  for (int j = wave; j < ninstr; j += NWAVE) {
    const int s = j * 64 + lane;
    const int row = s / CPR, c = swz(row, s % CPR);
    __builtin_amdgcn_global_load_lds(g + (row0 + row) * kp_bytes + k0_bytes + 16 * c, l + j * 1024, 16, 0, 0);
  }
}

template <int TM>
__global__ __launch_bounds__(256, 1) void exchange_big_kernel(ExchBigArgs g) {
  using G = Geo<TM>;
  constexpr int R = G::ROWS;
  __shared__ __align__(16) unsigned char lds0[G::SIZE];
  __shared__ __align__(16) unsigned char lds1[G::SIZE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  const long kpb = (long)g.kp * 2;
  const int rows = g.rows;                        // rows loaded per region and plane (<= R)

  f4 acc[TM][TM];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  auto issue = [&](int chunk, unsigned char* buf) {
    const long k0b = (long)chunk * KC * 2;
    lds_t* l = (lds_t*)buf;
    dma_region(static_cast<const unsigned char*>(g.a[0]), arow0, kpb, k0b, l, rows, wave, lane);
    dma_region(static_cast<const unsigned char*>(g.a[1]), arow0, kpb, k0b, l + R * ROWB, rows, wave, lane);
    dma_region(static_cast<const unsigned char*>(g.b[0]), brow0, kpb, k0b, l + 2 * R * ROWB, rows, wave, lane);
    dma_region(static_cast<const unsigned char*>(g.b[1]), brow0, kpb, k0b, l + 3 * R * ROWB, rows, wave, lane);
  };

  const int nchunk = g.kp / KC;                   // even
  const int arow = nb * N, brow = part * N;       // this wave's first rows in the A / B regions
  issue(0, lds0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int c = 0; c < nchunk; c += 2) {
    issue(c + 1, lds1);
    mma_chunk<TM>(acc, lds0, lds0 + 2 * R * ROWB, arow, brow, lane);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (c + 2 < nchunk) issue(c + 2, lds0);
    mma_chunk<TM>(acc, lds1, lds1 + 2 * R * ROWB, arow, brow, lane);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }

  // ---- epilogue: both planes of each block in LDS (row stride N + 1) ----
  // tr(Omega Omega) = sum_a Omega_aa^2 + 2 sum_{a<b} Omega_ab Omega_ba: waves
  // store their lower-triangle tiles (i >= j) and read the transposed partners
  // of their upper-triangle tiles (i <= j). Branch-free: out-of-range lanes
  // store to a private trash slot and read a clamped address with a zero
  // weight. Products of the FP32 accumulators are formed in FP64 (exact).
  __shared__ float trash[NWAVE * 64];
  const int S = N + 1;
  float* pl = reinterpret_cast<float*>(nb == 0 ? lds0 : lds1);
  float* mine = pl + part * N * S;
  const float* other = pl + (part ^ 1) * N * S;
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
        const bool ok = (i < TM - 1 || a < N) && (j < TM - 1 || b < N);
        float* dst = ok ? mine + a * S + b : my_trash;
        *dst = acc[i][j][r];
      }
    }
  __syncthreads();
  double s[5] = {0, 0, 0, 0, 0};   // tr_re, tr_im, rere, imim, reim
  double d_diag = 0.0, d_same = 0.0, d_other = 0.0;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = i; j < TM; ++j) {
      const int b = 16 * j + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * i + 4 * lq + r;
        const bool ok = (i < TM - 1 || a < N) && (j < TM - 1 || b < N);
        const int idx = ok ? b * S + a : 0;
        const double v = ok ? (double)acc[i][j][r] : 0.0;
        const double ps = mine[idx], po = other[idx];
        if (i < j) {                       // whole tile above the diagonal: a < b
          d_same += 2.0 * v * ps;
          d_other += v * po;
        } else {
          const double ws = a < b ? 2.0 : (a == b ? 1.0 : 0.0);
          const double wo = a < b ? 1.0 : ((a == b && part == 0) ? 1.0 : 0.0);
          d_same += ws * v * ps;
          d_other += wo * v * po;
          d_diag += a == b ? v : 0.0;
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
  constexpr int R = Geo<TM>::ROWS;
  g.rows = round_up(g.n + 16 * TM, 16);
  AFQ_CHECK(g.rows <= R && g.n <= 16 * TM, AFQ_E_INVALID, "exchange: tile does not cover the block");
  AFQ_CHECK(g.kp % (2 * KC) == 0, AFQ_E_INVALID, "exchange: contraction length must be a multiple of 64");
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
