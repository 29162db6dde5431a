// FP32 contractions of the reduced-precision modes on v_mfma_f32_16x16x4f32,
// streamed through the three-stage direct global->LDS ring:
//
//   * the propagator matrices A_w = sum_n c_wn L^n: coefficient rows
//     (w, Re|Im) times the upper block triangle of the symmetric Cholesky
//     vectors (8 x 8 block pairs, half the M^2 columns), packed once per system
//     k-contiguous (entry e at [n / 16][e][n % 16]); the epilogue writes each
//     block of the complex symmetric A_w and its mirror in real form, rows
//     (m, Re) = [Re A, -Im A] and (m, Im) = [Im A, Re A] interleaved over k,
//     packed k-contiguous for the Taylor products;
//   * the Taylor propagator in Horner form, U = V + A (V + A/2 (... (V + A V/K))),
//     V = B1 W: every product is the real contraction of the walker columns
//     (rows n of the packed term, Re/Im interleaved over k) with the real form
//     of A, so row n of the output is [Re, Im] of (A h)[m][n] over columns
//     2m + part; intermediate terms V + A h / j stay FP32 in the packed layout,
//     the last one is added to V in FP64;
//   * the products B1 W and B1 U of the propagator as W + (B1 - I) W: the
//     correction (B1 - I = O(dt h')) in FP32, walker rows (n, Re|Im) against
//     rows m of B1 - I, added to W in FP64, so the product keeps FP64-class
//     accuracy;
//   * the force-bias traces tr(Lt^{ns} Theta^s) = sum_(a,k) Theta-hat[(a,k)] Lt_n[a][k]
//     (split-BF16x3 mode, real trial): Theta-hat rows (w, Re|Im) times the
//     real half-rotated vectors, packed once per system; the N M contraction is
//     split into runs whose FP32 tiles are summed in FP64 in a fixed order.
//
// All are C = A B^T with A and B packed chunk-major (64-byte rows of 16 FP32
// contraction elements, all rows of a chunk contiguous), the layout and
// swizzle of the split-BF16x3 kernels, batched over walkers where the
// operands are per walker. Two tile geometries: 256 x 128 (2 x 2 waves of
// 8 x 4 MFMA tiles) for the propagator build and the force bias, 224 x 160
// (7 x 5 tiles) for the Taylor products, whose n_tot walker columns and 2M
// real-form rows it covers with little padding at the M = 400, N = 200 shape.
// 72-74 KB of LDS, two workgroups per CU.
//
// In split-BF16x3 mode the Horner products run on v_mfma_f32_16x16x32_bf16
// instead (hi*hi + hi*lo + lo*hi, FP32 accumulation; the shared chunk loop
// of mfma_ring.h): the propagator build writes A in compact form as BF16 hi /
// lo planes (rows m = [Re A, Im A] over k, the products form the real-form
// rows in registers), and each product's epilogue adds V (FP32) and splits
// the next term into hi / lo planes. Every term is multiplied by A again
// before it reaches U, and |A| is small (O(sqrt(dt)) per Cholesky vector), so
// the BF16 products' rounding reaches U damped by |A|; the last product is
// still added to V in FP64.
#include <algorithm>
#include <vector>
#include <type_traits>
#include "common.h"
#include "mfma_ring.h"

namespace {

using ring::f4;
using ring::lds_t;
using ring::ROWB;
using ring::swz;
using ring::wait_vm_barrier;

constexpr int NWAVE = 4, NXCD = 8;
constexpr int RK = 16;   // FP32 contraction elements per chunk row

template <int TA_, int TB_> struct Geo {
  static constexpr int TA = TA_, TB = TB_;
  static constexpr int RA = 32 * TA, RB = 32 * TB;
  static constexpr int REGA = RA * ROWB, REGB = RB * ROWB, STAGE = REGA + REGB;
  static constexpr int NT = STAGE / 1024, NQ = NT / NWAVE;
  static_assert(NT % NWAVE == 0, "loads must split evenly over the waves");
};
using GeoAB = Geo<8, 4>;   // propagator build, force bias
using GeoTY = Geo<7, 5>;   // Taylor products

enum { EPI_XFORM = 0, EPI_PART = 1, EPI_HORNER = 2, EPI_B1 = 3, EPI_HORNER_LAST = 5 };

// split BF16 of an FP32 value: hi = bf16(f), lo = bf16(f - hi), both rounded
// to nearest even; a pair (x, y) of them packed as two BF16 (x low) per plane
__device__ inline unsigned bf16_bits(float f) {
  const unsigned u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline void split_pair(float x, float y, unsigned& hi, unsigned& lo) {
  const unsigned xh = bf16_bits(x), yh = bf16_bits(y);
  const unsigned xl = bf16_bits(x - __uint_as_float(xh << 16)), yl = bf16_bits(y - __uint_as_float(yh << 16));
  hi = xh | (yh << 16);
  lo = xl | (yl << 16);
}

struct R32Args {
  const unsigned char* a;   // packed A: [chunk][rows_a][16] float (per batch member at a_bstride bytes)
  const unsigned char* b;   // packed B: [chunk][rows_b][16] float
  long rows_a, rows_b, a_bstride, b_bstride;
  int nchunk, kper, nblk_a, nblk_b, nbatch;
  int nunit, grid;          // units = A row blocks x contraction runs; grid = batch x units x B blocks
  int a_fast;               // 1: consecutive workgroups take consecutive A row blocks (sharing a B block)
  // EPI_XFORM: A rows (w, Re|Im), B rows e = 64 p + 8 mi + ki of block pair p = (bm, bk)
  // (tri[p] = bm << 16 | bk): m = 8 bm + mi, k = 8 bk + ki -> real form of A_w at
  // x + w x_wstride, at (m, k) and, off the diagonal blocks, at (k, m)
  const int* tri;
  float* x;
  long x_wstride, x_rows, ncol;
  int M, nw;
  // EPI_PART: part[(run * rows_a + row) * rows_b + col]
  float* part;
  // EPI_HORNER(_LAST): A rows n (walker columns), B rows 2m + part; batch member = walker
  const float* vy;          // V in the packed term layout
  float* yout;              // V + scale (A h) in the packed term layout (intermediate terms)
  double2* u;               // U[w][m][n] += scale (A h) (last term)
  float scale;
  long y_rows, y_wstride;
  int ntot;
  // EPI_B1: A rows (n, Re|Im) of a walker, B rows m of (B1 - I):
  // u[w][m][n] = ubase[w][m][n] + ((B1 - I) W)[m][n]
  const double2* ubase;
};

template <class G, int EPI>
__global__ __launch_bounds__(256, 2) void ring32_kernel(R32Args g) {
  constexpr int TA = G::TA, TB = G::TB, RA = G::RA, RB = G::RB, REGA = G::REGA, NQ = G::NQ;
  __shared__ __align__(16) unsigned char L0[G::STAGE];
  __shared__ __align__(16) unsigned char L1[G::STAGE];
  __shared__ __align__(16) unsigned char L2[G::STAGE];
  __shared__ float trash[NWAVE * 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rb = wave >> 1, cb = wave & 1;
  // XCD-aware order: workgroup i runs on XCD i % 8; each XCD takes a
  // contiguous range of the logical order
  const int per = (int)(gridDim.x / NXCD);
  const int lid = (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
  if (lid >= g.grid) return;
  int u, bb, batch;
  if (g.a_fast) {
    u = lid % g.nunit;
    const int rest = lid / g.nunit;
    bb = rest % g.nblk_b;
    batch = rest / g.nblk_b;
  } else {
    bb = lid % g.nblk_b;
    const int rest = lid / g.nblk_b;
    u = rest % g.nunit;
    batch = rest / g.nunit;
  }
  const int p = u % g.nblk_a, run = u / g.nblk_a;
  const int c0 = run * g.kper, nc = min(g.kper, g.nchunk - c0);   // >= 1
  const long arow0 = (long)p * RA, brow0 = (long)bb * RB;
  const unsigned char* abase = g.a + batch * g.a_bstride;
  const unsigned char* bbase = g.b + batch * g.b_bstride;
  // load q of this wave: instruction t = q * 4 + wave of the stage, 16 rows of
  // A (t < RA / 16) or B; lane l writes LDS bytes 1024 t + 16 l (row l / 4, swizzled piece)
  const unsigned char* src[NQ];
  long cstride[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = q * NWAVE + wave;
    const bool isb = t >= RA / 16;
    const int j = isb ? t - RA / 16 : t;
    const int row = 16 * j + (lane >> 2), c = swz(row, lane & 3);
    cstride[q] = (isb ? g.rows_b : g.rows_a) * (long)ROWB;
    src[q] = (isb ? bbase : abase) + ((isb ? brow0 : arow0) + row) * ROWB + 16 * c + (long)c0 * cstride[q];
  }
  auto issue = [&](int chunk, unsigned char* buf) {
    lds_t* l = (lds_t*)buf;
#pragma unroll
    for (int q = 0; q < NQ; ++q) ring::dma16(src[q] + chunk * cstride[q], l + (q * NWAVE + wave) * 1024);
  };
  // the last two steps have no chunk to prefetch: tiny loads into this wave's
  // trash slice keep the wait count of every step the same
  auto issue_dummy = [&]() {
    lds_t* l = (lds_t*)(trash + wave * 64);
#pragma unroll
    for (int q = 0; q < NQ; ++q) ring::dma4(src[q], l);
  };
  f4 acc[TA][TB];
#pragma unroll
  for (int i = 0; i < TA; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int arow = rb * (RA / 2), brow = cb * (RB / 2);
  issue(0, L0);
  if (nc > 1) issue(1, L1);
  else issue_dummy();
  wait_vm_barrier<NQ>();
  // step c: prefetch chunk c+2 into the buffer chunk c-1 used, multiply chunk
  // c, wait until chunk c+1 has landed (buffers rotated, one step per chunk)
  unsigned char* cur = L0;
  unsigned char* nxt = L1;
  unsigned char* pf = L2;
  for (int c = 0; c < nc; ++c) {
    if (c + 2 < nc) issue(c + 2, pf);
    else issue_dummy();
    __builtin_amdgcn_sched_barrier(0);
    ring::mma_f32<TA, TB>(acc, cur, cur + REGA, arow, brow, lane);
    __builtin_amdgcn_sched_barrier(0);
    wait_vm_barrier<NQ>();
    unsigned char* t = cur;
    cur = nxt;
    nxt = pf;
    pf = t;
  }
  wait_vm_barrier<0>();

  // lane (lr, lq) holds rows 4 lq .. 4 lq + 3 of column lr of every tile
  const int lr = lane & 15, lq = lane >> 4;
  if constexpr (EPI == EPI_XFORM) {
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        const long row0 = arow0 + arow + 16 * i + 4 * lq;    // rows (w0, Re), (w0, Im), (w0 + 1, Re), (w0 + 1, Im)
        const long col = brow0 + brow + 16 * j + lr;
        if (col >= g.ncol) continue;
        // a wave's 64 columns are one block pair: the direct stores of 8
        // neighbouring lanes fill one 64-byte packed row, the mirrored ones
        // fill theirs over the wave's four column tiles
        const int code = g.tri[col >> 6], bm = code >> 16, bk = code & 0xffff;
        const int m = 8 * bm + (int)((col >> 3) & 7), k = 8 * bk + (int)(col & 7);
        if (m >= g.M || k >= g.M) continue;
        const long o0 = ((long)(k >> 3) * g.x_rows + 2 * m) * RK + 2 * (k & 7);
        const long o1 = ((long)(m >> 3) * g.x_rows + 2 * k) * RK + 2 * (m & 7);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int w = (int)(row0 >> 1) + h;
          if (w < g.nw) {
            const float ar = acc[i][j][2 * h], ai = acc[i][j][2 * h + 1];
            float* X = g.x + (long)w * g.x_wstride;
            *reinterpret_cast<float2*>(X + o0) = make_float2(ar, -ai);
            *reinterpret_cast<float2*>(X + o0 + RK) = make_float2(ai, ar);
            if (bm != bk) {
              *reinterpret_cast<float2*>(X + o1) = make_float2(ar, -ai);
              *reinterpret_cast<float2*>(X + o1 + RK) = make_float2(ai, ar);
            }
          }
        }
      }
  } else if constexpr (EPI == EPI_PART) {
    float* out = g.part + (long)run * g.rows_a * g.rows_b;
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
      for (int j = 0; j < TB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const long row = arow0 + arow + 16 * i + 4 * lq + v;
          const long col = brow0 + brow + 16 * j + lr;
          out[row * g.rows_b + col] = acc[i][j][v];
        }
  } else if constexpr (EPI == EPI_B1) {
    // per row tile: gather every U_base value, then add and store (the loads
    // are not held back behind the stores, which the compiler cannot tell
    // apart from them)
#pragma unroll
    for (int i = 0; i < TA; ++i) {
      const long n0 = (arow0 + arow + 16 * i + 4 * lq) >> 1;   // rows (n0, Re), (n0, Im), (n0 + 1, Re), (n0 + 1, Im)
      double2 v[TB][2];
      long idx[TB][2];
      bool ok[TB][2];
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        const long m = brow0 + brow + 16 * j + lr;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const long n = n0 + h;
          ok[j][h] = m < g.M && n < g.ntot;
          idx[j][h] = ok[j][h] ? ((long)batch * g.M + m) * g.ntot + n : 0;
          v[j][h] = g.ubase[idx[j][h]];
        }
      }
#pragma unroll
      for (int j = 0; j < TB; ++j)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (ok[j][h])
            g.u[idx[j][h]] = make_double2(v[j][h].x + (double)acc[i][j][2 * h], v[j][h].y + (double)acc[i][j][2 * h + 1]);
    }
  } else {
    // column 2m + part of row n is part (Re, Im) of (A h)[m][n]: the partner
    // lane lr ^ 1 holds the other part; even lanes finish rows 0, 1 of their
    // four, odd lanes rows 2, 3. Per row tile every input is gathered before
    // any output is stored.
    const bool odd = lr & 1;
#pragma unroll
    for (int i = 0; i < TA; ++i) {
      const long n0 = arow0 + arow + 16 * i + 4 * lq;
      float re[TB][2], im[TB][2];
      long idx[TB][2];
      bool ok[TB][2];
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        float o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = __shfl_xor(acc[i][j][r], 1);
        const int col = (int)(brow0 + brow + 16 * j + lr), m = col >> 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const long n = n0 + (odd ? 2 + h : h);
          re[j][h] = odd ? o[2 + h] : acc[i][j][h];
          im[j][h] = odd ? acc[i][j][2 + h] : o[h];
          ok[j][h] = n < g.ntot && m < g.M;
          if constexpr (EPI == EPI_HORNER_LAST)
            idx[j][h] = ok[j][h] ? ((long)batch * g.M + m) * g.ntot + n : 0;
          else
            idx[j][h] = ok[j][h] ? (long)batch * g.y_wstride + ((long)(m >> 3) * g.y_rows + n) * RK + 2 * (m & 7) : 0;
        }
      }
      if constexpr (EPI == EPI_HORNER_LAST) {
        double2 v[TB][2];
#pragma unroll
        for (int j = 0; j < TB; ++j)
#pragma unroll
          for (int h = 0; h < 2; ++h) v[j][h] = g.u[idx[j][h]];
#pragma unroll
        for (int j = 0; j < TB; ++j)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (ok[j][h])
              g.u[idx[j][h]] = make_double2(v[j][h].x + (double)(g.scale * re[j][h]), v[j][h].y + (double)(g.scale * im[j][h]));
      } else {
        float2 v[TB][2];
#pragma unroll
        for (int j = 0; j < TB; ++j)
#pragma unroll
          for (int h = 0; h < 2; ++h) v[j][h] = *reinterpret_cast<const float2*>(g.vy + idx[j][h]);
#pragma unroll
        for (int j = 0; j < TB; ++j)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (ok[j][h])
              *reinterpret_cast<float2*>(g.yout + idx[j][h]) =
                  make_float2(v[j][h].x + g.scale * re[j][h], v[j][h].y + g.scale * im[j][h]);
      }
    }
  }
}

// Products of split-BF16x3 mode on the BF16 ring, both operands as BF16
// hi / lo planes of 32-element chunks, [chunk][rows][32] per plane, a walker's
// hi plane then its lo plane:
//   * B3_HORNER(_LAST): the contraction of EPI_HORNER (walker columns h, rows n,
//     against the real form of A, rows 2m + part, formed in registers from
//     the compact rows m = [Re A, Im A] that are stored);
//   * B3_B1: the contraction of EPI_B1 (walker rows (n, Re|Im) against the rows
//     m of B1 - I, shared by all walkers: b_wstride 0), added to U_base in FP64;
//   * B3_XFORM: the propagator build (coefficient rows against the upper block
//     triangle of L, one batch; consecutive workgroups take consecutive
//     coefficient row blocks, so they share an L block in L2), A_w written in
//     compact form (rows m = [Re A, Im A] over k) as BF16 hi / lo planes.
struct HornerB3Args {
  const unsigned char* a;   // terms h: rows n, contraction 2m + part
  const unsigned char* b;   // A in compact form, rows m (Horner), or B1 - I (rows m)
  long rows_a, rows_b, a_plane, b_plane, a_wstride, b_wstride;   // bytes (planes, walkers)
  int nchunk, nblk_a, nblk_b, nw, grid;
  const float* vy;          // V in the FP32 packed term layout (16-element chunks)
  long vy_rows, vy_wstride; // its rows and walker stride (floats)
  unsigned char* yout;      // V + scale (A h), laid out as a (intermediate terms)
  double2* u;               // U[w][m][n] += scale (A h) (last term); B3_B1: U = U_base + (B1 - I) W
  const double2* ubase;
  float scale;
  int ntot, M;
  // B3_XFORM: coefficient rows (w, Re|Im) against the block-pair columns of L
  // (tri, ncol); A_w in compact form to BF16 planes x (x_rows rows, x_plane
  // bytes apart, walkers x_wstride bytes apart)
  const int* tri;
  unsigned char* x;
  long x_rows, x_plane, x_wstride, ncol;
  // B3_B1, optional: the new U also as V of the Taylor products, in the FP32
  // packed term layout (vp) and as BF16 term planes (vb, laid out as yout)
  float* vp;
  long vp_rows, vp_wstride;
  unsigned char* vb;
  long vb_rows, vb_plane, vb_wstride;
  // B3_HORNER_LAST, optional: the new U also as the walker rows of the B1
  // product that follows (BF16 hi / lo planes, the layout of
  // pack_walker_rows_bf3_kernel), so that it needs no packing pass
  unsigned char* wr;
  long wr_rows, wr_plane, wr_wstride;
};

enum { B3_HORNER = 0, B3_HORNER_LAST = 1, B3_B1 = 2, B3_XFORM = 3 };

template <int TA, int TB, int MODE>
__global__ __launch_bounds__(256, 1) void horner_bf3_kernel(HornerB3Args g) {
  constexpr bool LAST = MODE != B3_HORNER;   // the input is U (or U_base): FP64
  // the Horner products read A_w in compact form (half the rows, see bf3_stream)
  constexpr bool CB = MODE == B3_HORNER || MODE == B3_HORNER_LAST;
  constexpr int RA = 32 * TA, RB = 32 * TB, RBS = CB ? RB / 2 : RB;   // RBS: stored B rows per tile
  constexpr int REGA = RA * ROWB, REGB = RBS * ROWB;
  // loads: A hi, A lo, B hi, B lo, then padding to a multiple of the waves
  // (extra loads fetch B rows again into the padding of the stage)
  constexpr int NTR = (2 * REGA + 2 * REGB) / 1024, NT = (NTR + NWAVE - 1) / NWAVE * NWAVE, NQ = NT / NWAVE;
  constexpr int STAGE = NT * 1024;
  constexpr int QA = (RA / 8) / NWAVE;        // the first QA loads of every wave move A rows
  static_assert((RA / 8) % NWAVE == 0, "A loads must split evenly over the waves");
  __shared__ __align__(16) unsigned char L0[STAGE];
  __shared__ __align__(16) unsigned char L1[STAGE];
  __shared__ __align__(16) unsigned char L2[STAGE];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar address arithmetic
  const int rb = wave >> 1, cb = wave & 1;
  // XCD-aware order: workgroup i runs on XCD i % 8; each XCD takes a
  // contiguous range of the logical order (B blocks fastest, so the blocks of
  // one walker share its terms in that XCD's L2)
  const int per = (int)(gridDim.x / NXCD);
  const int lid = (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
  if (lid >= g.grid) return;
  int bb, p, w;
  if constexpr (MODE == B3_XFORM) {
    p = lid % g.nblk_a;
    bb = (lid / g.nblk_a) % g.nblk_b;
    w = 0;
  } else {
    bb = lid % g.nblk_b;
    const int rest = lid / g.nblk_b;
    p = rest % g.nblk_a;
    w = rest / g.nblk_a;
  }
  const long arow0 = (long)p * RA, brow0 = (long)bb * RB;
  const unsigned char* abase = g.a + (long)w * g.a_wstride;
  const unsigned char* bbase = g.b + (long)w * g.b_wstride;
  // load q of this wave: instruction t = q * 4 + wave of the stage, 16 rows of
  // one region (A hi, A lo, B hi, B lo) starting at row 16 j of the region
  ring::StrideLoader<NQ, QA> ld;
  ld.astride = g.rows_a * (long)ROWB;
  ld.bstride = g.rows_b * (long)ROWB;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = q * NWAVE + wave;
    const int tt = t < NTR ? t : RA / 8;      // padding loads: B hi rows again
    const int reg = tt < RA / 16 ? 0 : tt < RA / 8 ? 1 : tt < RA / 8 + RBS / 16 ? 2 : 3;
    const int j = reg == 0 ? tt : reg == 1 ? tt - RA / 16 : reg == 2 ? tt - RA / 8 : tt - RA / 8 - RBS / 16;
    const unsigned char* base = reg == 0 ? abase : reg == 1 ? abase + g.a_plane : reg == 2 ? bbase : bbase + g.b_plane;
    ld.qb[q] = base + ((q < QA ? arow0 : (long)bb * RBS) + 16 * j) * ROWB;
  }
  f4 acc[TA][TB];
#pragma unroll
  for (int i = 0; i < TA; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int arow = rb * (RA / 2), brow = cb * (RB / 2);
  ring::bf3_stream<TA, TB, REGA, REGB, NQ, CB>(acc, (const lds_t*)L0, (const lds_t*)L1, (const lds_t*)L2,
                                               g.nchunk, arow, brow, lane, wave, ld);

  if constexpr (MODE == B3_XFORM) {
    // rows (w0, Re), (w0, Im), (w0 + 1, Re), (w0 + 1, Im); a wave's 64 columns
    // are one block pair (m in block bm, k in block bk): A_w[m][k] and, off the
    // diagonal blocks, its mirror A_w[k][m], in compact form: row m = [.., ar,
    // ai, ..] at elements 2k, 2k + 1 (the Horner products form the real-form
    // rows (m, Re) = [ar, -ai] and (m, Im) = [ai, ar] from it in registers)
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        const long row0 = arow0 + arow + 16 * i + 4 * lq;
        const long col = brow0 + brow + 16 * j + lr;
        if (col >= g.ncol) continue;
        const int code = g.tri[col >> 6], bm = code >> 16, bk = code & 0xffff;
        const int m = 8 * bm + (int)((col >> 3) & 7), k = 8 * bk + (int)(col & 7);
        if (m >= g.M || k >= g.M) continue;
        const long b0 = ((long)(k >> 4) * g.x_rows + m) * ROWB + 4 * (k & 15);
        const long b1 = ((long)(m >> 4) * g.x_rows + k) * ROWB + 4 * (m & 15);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int wk = (int)(row0 >> 1) + h;
          if (wk < g.nw) {
            const float ar = acc[i][j][2 * h], ai = acc[i][j][2 * h + 1];
            unsigned char* X = g.x + (long)wk * g.x_wstride;
            unsigned ch, cl;
            split_pair(ar, ai, ch, cl);
            *reinterpret_cast<unsigned*>(X + b0) = ch;
            *reinterpret_cast<unsigned*>(X + g.x_plane + b0) = cl;
            if (bm != bk) {
              *reinterpret_cast<unsigned*>(X + b1) = ch;
              *reinterpret_cast<unsigned*>(X + g.x_plane + b1) = cl;
            }
          }
        }
      }
    return;
  }
  // column 2m + part of row n is part (Re, Im) of (A h)[m][n]: the partner
  // lane lr ^ 1 holds the other part; even lanes finish rows 0, 1 of their
  // four, odd lanes rows 2, 3. The inputs of row tile i + 1 (V, or U for the
  // last term) are loaded before the outputs of row tile i are stored, so
  // only the first tile waits a full memory round trip.
  const int lr = lane & 15, lq = lane >> 4;
  const bool odd = lr & 1;
  using In = typename std::conditional<LAST, double2, float2>::type;
  auto at = [&](int i, int j, int h, bool& ok) -> long {
    if constexpr (MODE == B3_B1) {   // rows (n0, Re), (n0, Im), (n0 + 1, Re), (n0 + 1, Im); column m
      const long n = ((arow0 + arow + 16 * i + 4 * lq) >> 1) + h;
      const long m = brow0 + brow + 16 * j + lr;
      ok = n < g.ntot && m < g.M;
      return ok ? ((long)w * g.M + m) * g.ntot + n : 0;
    }
    const long n = arow0 + arow + 16 * i + 4 * lq + (odd ? 2 + h : h);
    const int m = (int)((brow0 + brow + 16 * j + lr) >> 1);
    ok = n < g.ntot && m < g.M;
    if (!ok) return 0;
    if constexpr (LAST) return ((long)w * g.M + m) * g.ntot + n;
    else return (long)w * g.vy_wstride + ((long)(m >> 3) * g.vy_rows + n) * RK + 2 * (m & 7);
  };
  auto load = [&](long idx) -> In {
    if constexpr (MODE == B3_B1) return g.ubase[idx];
    else if constexpr (LAST) return g.u[idx];
    else return *reinterpret_cast<const float2*>(g.vy + idx);
  };
  In pre[TB][2];
#pragma unroll
  for (int j = 0; j < TB; ++j)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bool ok;
      pre[j][h] = load(at(0, j, h, ok));
    }
#pragma unroll
  for (int i = 0; i < TA; ++i) {
    In cur[TB][2];
#pragma unroll
    for (int j = 0; j < TB; ++j)
#pragma unroll
      for (int h = 0; h < 2; ++h) cur[j][h] = pre[j][h];
    if (i + 1 < TA) {
#pragma unroll
      for (int j = 0; j < TB; ++j)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          bool ok;
          pre[j][h] = load(at(i + 1, j, h, ok));
        }
    }
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      if constexpr (MODE == B3_B1) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          bool ok;
          const long idx = at(i, j, h, ok);
          if (!ok) continue;
          const double2 nv = make_double2(cur[j][h].x + (double)acc[i][j][2 * h], cur[j][h].y + (double)acc[i][j][2 * h + 1]);
          g.u[idx] = nv;
          if (g.vp) {
            const long n = ((arow0 + arow + 16 * i + 4 * lq) >> 1) + h;
            const long m = brow0 + brow + 16 * j + lr;
            const float2 f = make_float2((float)nv.x, (float)nv.y);
            *reinterpret_cast<float2*>(g.vp + (long)w * g.vp_wstride + ((m >> 3) * g.vp_rows + n) * RK + 2 * (m & 7)) = f;
            unsigned hi, lo;
            split_pair(f.x, f.y, hi, lo);
            unsigned char* y = g.vb + (long)w * g.vb_wstride + ((m >> 4) * g.vb_rows + n) * ROWB + 4 * (m & 15);
            *reinterpret_cast<unsigned*>(y) = hi;
            *reinterpret_cast<unsigned*>(y + g.vb_plane) = lo;
          }
        }
        continue;
      }
      float o[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r] = __shfl_xor(acc[i][j][r], 1);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float re = odd ? o[2 + h] : acc[i][j][h], im = odd ? acc[i][j][2 + h] : o[h];
        bool ok;
        const long idx = at(i, j, h, ok);
        if constexpr (LAST) {
          const double2 nv = make_double2(cur[j][h].x + (double)(g.scale * re), cur[j][h].y + (double)(g.scale * im));
          if (ok) g.u[idx] = nv;
          if (g.wr) {
            // walker rows (n, Re|Im) over m: lane lr holds m = col / 2, lane
            // lr ^ 2 (same quad, same rows n) holds m ^ 1. The pair (even m,
            // m + 1) is split as the packing kernel splits it; the lane of the
            // even m writes its real parts, the other lane its imaginary parts
            // (k >= M and rows past n_tot read as zero there too)
            const float fx = ok ? (float)nv.x : 0.f, fy = ok ? (float)nv.y : 0.f;
            const bool em = !(lr & 2);
            const float mine = em ? fx : fy, other = em ? fy : fx;   // this lane's part, the partner's
            const float pv = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(other), 0x4E, 0xf, 0xf, false));
            const long n = arow0 + arow + 16 * i + 4 * lq + (odd ? 2 + h : h);
            const int m0 = (int)((brow0 + brow + 16 * j + lr) >> 1) & ~1;   // the even m of the pair
            if (n < g.ntot && m0 < g.M) {
              unsigned char* y = g.wr + (long)w * g.wr_wstride +
                                 ((long)(m0 >> 5) * g.wr_rows + 2 * n + (em ? 0 : 1)) * ROWB + 2 * (m0 & 31);
              unsigned hi, lo;
              split_pair(em ? mine : pv, em ? pv : mine, hi, lo);
              *reinterpret_cast<unsigned*>(y) = hi;
              *reinterpret_cast<unsigned*>(y + g.wr_plane) = lo;
            }
          }
        } else {
          if (!ok) continue;
          const long n = arow0 + arow + 16 * i + 4 * lq + (odd ? 2 + h : h);
          const int m = (int)((brow0 + brow + 16 * j + lr) >> 1);
          unsigned hi, lo;
          split_pair(cur[j][h].x + g.scale * re, cur[j][h].y + g.scale * im, hi, lo);
          unsigned char* y = g.yout + (long)w * g.a_wstride + ((long)(m >> 4) * g.rows_a + n) * ROWB + 4 * (m & 15);
          *reinterpret_cast<unsigned*>(y) = hi;
          *reinterpret_cast<unsigned*>(y + g.a_plane) = lo;
        }
      }
    }
  }
}

// W[w][k][n] (complex FP64) -> BF16 hi / lo planes of walker rows (n, Re|Im):
// component part of W[k][n] at ((k / 32) rows + 2n + part) 64 + 2 (k % 32)
// bytes, zero for k >= M. A workgroup moves a 32 (k) x 8 (n) tile through LDS;
// each of its 16 rows is written as 64 contiguous bytes per plane.
__global__ __launch_bounds__(256) void pack_walker_rows_bf3_kernel(const double2* __restrict__ W, int M, int ntot,
                                                                   long rows, long plane, long wstride,
                                                                   unsigned char* __restrict__ out) {
  __shared__ float2 tile[32][9];
  const int t = threadIdx.x, n0 = blockIdx.x * 8, k0 = blockIdx.y * 32, w = blockIdx.z;
  {
    const int k = k0 + (t >> 3), n = n0 + (t & 7);
    float2 v = make_float2(0.f, 0.f);
    if (k < M && n < ntot) {
      const double2 d = W[((long)w * M + k) * ntot + n];
      v = make_float2((float)d.x, (float)d.y);
    }
    tile[t >> 3][t & 7] = v;
  }
  __syncthreads();
  const int r = t >> 4, kp = t & 15, j = r >> 1, part = r & 1, n = n0 + j;
  if (n < ntot) {
    const float2 a = tile[2 * kp][j], b = tile[2 * kp + 1][j];
    unsigned hi, lo;
    split_pair(part ? a.y : a.x, part ? b.y : b.x, hi, lo);
    unsigned char* y = out + (long)w * wstride + ((long)blockIdx.y * rows + 2 * n + part) * ROWB + 4 * kp;
    *reinterpret_cast<unsigned*>(y) = hi;
    *reinterpret_cast<unsigned*>(y + plane) = lo;
  }
}

// (B1 - I) as BF16 hi / lo planes of rows m: element k at ((k / 32) rows + m) 64 + 2 (k % 32) bytes
__global__ void pack_b1_bf3_kernel(const double* __restrict__ B1, int M, long rows, int nchunk, long plane,
                                   unsigned short* __restrict__ out) {
  const long total = (long)nchunk * rows * 32;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long c = e / (rows * 32), rem = e - c * rows * 32;
    const long m = rem / 32, k = c * 32 + (rem - m * 32);
    const float f = (m < M && k < M) ? (float)(B1[m * M + k] - (m == k ? 1.0 : 0.0)) : 0.f;
    const unsigned h = bf16_bits(f);
    out[e] = (unsigned short)h;
    out[plane / 2 + e] = (unsigned short)bf16_bits(f - __uint_as_float(h << 16));
  }
}

// complex FP32 rows -> BF16 hi / lo planes of real rows (2 r + part), zero
// outside: element k of row 2r + part (component part of src[r ld + k]) at
// short ((k / 32) rows + 2r + part) 32 + k % 32 of the hi plane (lo plane
// plane_s shorts later)
__global__ void pack_cplx_rows_bf3_kernel(const float* __restrict__ src, long ld, int nrow_c, long K, long rows,
                                          int nchunk, long plane_s, unsigned short* __restrict__ out) {
  const long total = (long)nchunk * rows * 32;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long c = e / (rows * 32), rem = e - c * rows * 32;
    const long r = rem / 32, k = c * 32 + (rem - r * 32);
    const float f = ((r >> 1) < nrow_c && k < K) ? src[2 * ((r >> 1) * ld + k) + (r & 1)] : 0.f;
    const unsigned h = bf16_bits(f);
    out[e] = (unsigned short)h;
    out[plane_s + e] = (unsigned short)bf16_bits(f - __uint_as_float(h << 16));
  }
}

// the block-pair columns e of the symmetrised L^k (as pack_tri_cols_kernel)
// as BF16 hi / lo planes: element k of row e at short ((k / 32) rows + e) 32 +
// k % 32 (lo plane plane_s shorts later)
__global__ void pack_tri_cols_bf3_kernel(const double* __restrict__ src, int M, int K, const int* __restrict__ tri,
                                         long ncol, long rows, int nchunk, long plane_s,
                                         unsigned short* __restrict__ out) {
  const long total = (long)nchunk * rows * 32;
  const long m2 = (long)M * M;
  for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    const long k = t / rows, e = t - k * rows;
    float f = 0.f;
    if (k < K && e < ncol) {
      const int code = tri[e >> 6];
      const int m = 8 * (code >> 16) + (int)((e >> 3) & 7), kk = 8 * (code & 0xffff) + (int)(e & 7);
      if (m < M && kk < M) f = (float)(0.5 * (src[k * m2 + (long)m * M + kk] + src[k * m2 + (long)kk * M + m]));
    }
    const long o = ((k / 32) * rows + e) * 32 + (k % 32);
    const unsigned h = bf16_bits(f);
    out[o] = (unsigned short)h;
    out[plane_s + o] = (unsigned short)bf16_bits(f - __uint_as_float(h << 16));
  }
}

// V[w][m][n] (complex FP64) -> the BF16 hi / lo term planes of walker w:
// element (n, 2m + part) at ((m / 16) rows + n) 64 + 4 (m % 16) + 2 part bytes.
// A workgroup moves a 16 (m) x 16 (n) tile through LDS so that the reads (along
// n) and the writes (16 consecutive m of one row: 64 bytes per plane) are
// contiguous.
__global__ __launch_bounds__(256) void pack_terms_bf3_kernel(const double2* __restrict__ V, int M, int ntot, long rows,
                                                             long plane, long wstride, unsigned char* __restrict__ out) {
  __shared__ float2 tile[16][17];
  const int t = threadIdx.x, n0 = blockIdx.x * 16, m0 = blockIdx.y * 16, w = blockIdx.z;
  {
    const int m = m0 + (t >> 4), n = n0 + (t & 15);
    float2 v = make_float2(0.f, 0.f);
    if (m < M && n < ntot) {
      const double2 d = V[((long)w * M + m) * ntot + n];
      v = make_float2((float)d.x, (float)d.y);
    }
    tile[t >> 4][t & 15] = v;
  }
  __syncthreads();
  const int n = n0 + (t >> 4), e = t & 15, m = m0 + e;
  if (m < M && n < ntot) {
    const float2 v = tile[e][t >> 4];
    unsigned hi, lo;
    split_pair(v.x, v.y, hi, lo);
    unsigned char* y = out + (long)w * wstride + ((long)(m0 >> 4) * rows + n) * ROWB + 4 * e;
    *reinterpret_cast<unsigned*>(y) = hi;
    *reinterpret_cast<unsigned*>(y + plane) = lo;
  }
}

// complex rows -> real rows (2 r + part) of a packed operand, zero outside:
// out[(c rows + r) 16 + kk] = component (r & 1) of src[(r >> 1) ld + 16 c + kk]
template <typename S>
__global__ void pack_cplx_rows_kernel(const S* __restrict__ src, long ld, int nrow_c, long K, long rows, int nchunk,
                                      float* __restrict__ out) {
  const long total = (long)nchunk * rows * RK;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long c = e / (rows * RK), rem = e - c * rows * RK;
    const long r = rem / RK, k = c * RK + (rem - r * RK);
    float v = 0.f;
    if ((r >> 1) < nrow_c && k < K) v = (float)src[2 * ((r >> 1) * ld + k) + (r & 1)];
    out[e] = v;
  }
}

// real rows of a packed operand: out[(c rows + r) 16 + kk] = src[r ld + 16 c + kk]
__global__ void pack_real_rows_kernel(const double* __restrict__ src, long ld, int nrow, long K, long rows, int nchunk,
                                      float* __restrict__ out) {
  const long total = (long)nchunk * rows * RK;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long c = e / (rows * RK), rem = e - c * rows * RK;
    const long r = rem / RK, k = c * RK + (rem - r * RK);
    out[e] = (r < nrow && k < K) ? (float)src[r * ld + k] : 0.f;
  }
}

// The 8 x 8 block pairs (bm, bk), bm <= bk, of an M x M symmetric matrix in
// row order: tri[p] = bm << 16 | bk
__global__ void tri_table_kernel(int nb, int nbp, int* __restrict__ tri) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= nbp) return;
  int bm = 0, r = p;
  while (r >= nb - bm) {
    r -= nb - bm;
    ++bm;
  }
  tri[p] = bm << 16 | (bm + r);
}

// the upper block triangle of the symmetric L^n as rows of a packed operand
// (k = vector index): row e = 64 p + 8 mi + ki of block pair p = (bm, bk) holds
// (L^k[m][kk] + L^k[kk][m]) / 2, m = 8 bm + mi, kk = 8 bk + ki, zero outside
__global__ void pack_tri_cols_kernel(const double* __restrict__ src, int M, int K, const int* __restrict__ tri,
                                     long ncol, long rows, int nchunk, float* __restrict__ out) {
  const long total = (long)nchunk * rows * RK;
  const long m2 = (long)M * M;
  for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    const long k = t / rows, e = t - k * rows;
    float v = 0.f;
    if (k < K && e < ncol) {
      const int code = tri[e >> 6];
      const int m = 8 * (code >> 16) + (int)((e >> 3) & 7), kk = 8 * (code & 0xffff) + (int)(e & 7);
      if (m < M && kk < M) v = (float)(0.5 * (src[k * m2 + (long)m * M + kk] + src[k * m2 + (long)kk * M + m]));
    }
    out[((k / RK) * rows + e) * RK + (k % RK)] = v;
  }
}

// V[w][m][n] (complex FP64) -> the packed term layout of walker w: element
// (n, 2m + part) at ((m / 8) y_rows + n) 16 + 2 (m % 8) + part. A workgroup
// moves an 8 (m) x 32 (n) tile through LDS so that both the reads (along n)
// and the writes (8 consecutive m of one packed row) are contiguous.
__global__ __launch_bounds__(256) void pack_terms_kernel(const double2* __restrict__ V, int M, int ntot, long y_rows,
                                                         long y_wstride, float* __restrict__ out) {
  __shared__ float2 tile[8][33];
  const int t = threadIdx.x, n0 = blockIdx.x * 32, m0 = blockIdx.y * 8, w = blockIdx.z;
  {
    const int m = m0 + (t >> 5), n = n0 + (t & 31);
    float2 v = make_float2(0.f, 0.f);
    if (m < M && n < ntot) {
      const double2 d = V[((long)w * M + m) * ntot + n];
      v = make_float2((float)d.x, (float)d.y);
    }
    tile[t >> 5][t & 31] = v;
  }
  __syncthreads();
  const int n = n0 + (t >> 3), e = t & 7, m = m0 + e;
  if (m < M && n < ntot)
    *reinterpret_cast<float2*>(out + (long)w * y_wstride + ((long)(m0 >> 3) * y_rows + n) * RK + 2 * e) =
        tile[e][t >> 3];
}

// W[w][k][n] (complex FP64) -> rows (n, Re|Im) of walker w, k-contiguous:
// component part of W[k][n] at ((k / 16) rows + 2n + part) 16 + k % 16, zero for
// k >= M. A workgroup moves a 16 (k) x 16 (n) tile through LDS.
__global__ __launch_bounds__(256) void pack_walker_rows_kernel(const double2* __restrict__ W, int M, int ntot, long rows,
                                                               long wstride, float* __restrict__ out) {
  __shared__ float2 tile[16][17];
  const int t = threadIdx.x, n0 = blockIdx.x * 16, k0 = blockIdx.y * 16, w = blockIdx.z;
  {
    const int k = k0 + (t >> 4), n = n0 + (t & 15);
    float2 v = make_float2(0.f, 0.f);
    if (k < M && n < ntot) {
      const double2 d = W[((long)w * M + k) * ntot + n];
      v = make_float2((float)d.x, (float)d.y);
    }
    tile[t >> 4][t & 15] = v;
  }
  __syncthreads();
  const int r = t >> 3, kp = t & 7, j = r >> 1, part = r & 1, n = n0 + j;
  if (n < ntot) {
    const float2 a = tile[2 * kp][j], b = tile[2 * kp + 1][j];
    *reinterpret_cast<float2*>(out + (long)w * wstride + (((long)(k0 >> 4) * rows + 2 * n + part) * RK) + 2 * kp) =
        part ? make_float2(a.y, b.y) : make_float2(a.x, b.x);
  }
}

// (B1 - I) as rows m, k-contiguous: out[((k / 16) rows + m) 16 + k % 16]
__global__ void pack_b1_kernel(const double* __restrict__ B1, int M, long rows, int nchunk, float* __restrict__ out) {
  const long total = (long)nchunk * rows * RK;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long c = e / (rows * RK), rem = e - c * rows * RK;
    const long m = rem / RK, k = c * RK + (rem - m * RK);
    out[e] = (m < M && k < M) ? (float)(B1[m * M + k] - (m == k ? 1.0 : 0.0)) : 0.f;
  }
}

// tro[w][spin][n] = sum over runs (fixed order) of (part[run][2w][n], part[run][2w + 1][n])
// (with both: the traces of the spin sum, written to spin 0, and zero to spin 1)
__global__ void coulomb_reduce_kernel(const float* __restrict__ part, int nrun, long rows_a, long rows_b, int nw,
                                      int X, int spin, int both, double2* __restrict__ tro) {
  const long t = blockIdx.x * 256L + threadIdx.x;
  if (t >= (long)nw * X) return;
  const int w = (int)(t / X), n = (int)(t - (long)w * X);
  double re = 0.0, im = 0.0;
  for (int r = 0; r < nrun; ++r) {
    const float* p = part + (long)r * rows_a * rows_b;
    re += (double)p[(2L * w) * rows_b + n];
    im += (double)p[(2L * w + 1) * rows_b + n];
  }
  tro[((long)w * 2 + spin) * X + n] = make_double2(re, im);
  if (both) tro[((long)w * 2 + 1) * X + n] = make_double2(0.0, 0.0);
}

// Theta-hat of the spin sum as real rows (w, Re|Im), k-contiguous:
// out[(c rows + r) 16 + kk] = component (r & 1) of src[(r >> 1) ld + k] + src[(r >> 1) ld + off1 + k]
__global__ void pack_cplx_rows_sum_kernel(const double* __restrict__ src, long ld, long off1, int nrow_c, long K,
                                          long rows, int nchunk, float* __restrict__ out) {
  const long total = (long)nchunk * rows * RK;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long c = e / (rows * RK), rem = e - c * rows * RK;
    const long r = rem / RK, k = c * RK + (rem - r * RK);
    float v = 0.f;
    if ((r >> 1) < nrow_c && k < K) {
      const long i = 2 * ((r >> 1) * ld + k) + (r & 1);
      v = (float)(src[i] + src[i + 2 * off1]);
    }
    out[e] = v;
  }
}

int grid_of(long total) { return (int)std::min<long>(std::max<long>((total + 255) / 256, 1), 1 << 20); }
long pad_to(long x, long m) { return (x + m - 1) / m * m; }

template <class G, int EPI>
int launch(R32Args& g, hipStream_t st) {
  g.nblk_a = (int)(g.rows_a / G::RA);
  g.nblk_b = (int)(g.rows_b / G::RB);
  if (g.nbatch < 1) g.nbatch = 1;
  const int nrun = (g.nchunk + g.kper - 1) / g.kper;
  const long nunit = (long)g.nblk_a * nrun, grid = nunit * g.nblk_b * g.nbatch;
  AFQ_CHECK(g.nchunk >= 1 && g.kper >= 1 && g.rows_a % G::RA == 0 && g.rows_b % G::RB == 0 && grid < (1L << 30),
            AFQ_E_INVALID, "FP32 ring contraction: bad shape");
  g.nunit = (int)nunit;
  g.grid = (int)grid;
  const long launch = (grid + NXCD - 1) / NXCD * NXCD;
  hipLaunchKernelGGL((ring32_kernel<G, EPI>), dim3((unsigned)launch), dim3(256), 0, st, g);
  return hip_status(hipGetLastError(), "FP32 ring contraction");
}

// rows of the coefficient operand and of the Theta-hat operand for nw walkers
long coef_rows(int nw) { return pad_to(2L * nw, GeoAB::RA); }

// runs of the force-bias contraction: about 2048 workgroups, runs of at least 16 chunks
int coulomb_kper(long nchunk, long rows_a, long rows_b) {
  const long tiles = (rows_a / GeoAB::RA) * (rows_b / GeoAB::RB);
  const long nrun = std::max<long>(1, std::min<long>(nchunk / 16, (2048 + tiles - 1) / tiles));
  return (int)((nchunk + nrun - 1) / nrun);
}

// columns of the propagator build: 64 per 8 x 8 block pair of the upper block triangle
struct TriCols {
  int nb, nbp;
  long ncol, rows;
};
TriCols tri_cols(afq_system s) {
  TriCols t;
  t.nb = ceil_div(s->M, 8);
  t.nbp = t.nb * (t.nb + 1) / 2;
  t.ncol = 64L * t.nbp;
  t.rows = pad_to(t.ncol, GeoAB::RB);
  return t;
}

bool taylor_b3(afq_system s) { return s->prec == AFQ_BF16X3; }

// Tiles of the split-BF16x3 Taylor and B1 products (TA x TB MFMA tiles of
// 16 x 16 per wave, 2 x 2 waves: 32 TA term rows x 32 TB output columns per
// workgroup). The large tile suits the M = 400 walker (n_tot = 200 columns,
// 2M = 800 real-form rows: 89% of its products useful); small systems waste
// most of it on padding (at M = 64, n_tot = 32: 11%), which the small tiles
// avoid at the price of more workgroups and operand reloads.
struct B3Tile {
  int ta, tb;
};
constexpr B3Tile kB3Tiles[] = {{7, 5}, {4, 4}, {2, 2}};
constexpr int kNumB3Tiles = 3;

// padded MFMA work of one step's products with tile t: six Horner products
// (n_tot term rows, 2M columns, contraction 2M) and two B1 products (2 n_tot
// walker rows, M columns, contraction M)
double b3_tile_work(afq_system s, int t) {
  const long ra = 32L * kB3Tiles[t].ta, rb = 32L * kB3Tiles[t].tb, M = s->M, n = s->ntot;
  return 6.0 * pad_to(n, ra) * pad_to(2 * M, rb) * pad_to(2 * M, 32) + 2.0 * pad_to(2 * n, ra) * pad_to(M, rb) * pad_to(M, 32);
}

}  // namespace

// the tile a system uses: its pinned one, else the one with the least padded
// work, a larger tile winning when it needs at most 10% more (fewer
// workgroups, each reloading its operands less often)
int b3_tile_of(afq_system s) {
  if (s->b3_tile >= 0) return s->b3_tile;
  int best = 0;
  double best_w = b3_tile_work(s, 0);
  for (int t = 1; t < kNumB3Tiles; ++t) {
    const double w = b3_tile_work(s, t);
    if (w * 1.1 < best_w) {
      best = t;
      best_w = w;
    }
  }
  return best;
}
int b3_num_tiles() { return kNumB3Tiles; }

namespace {

// packed real form of A_w (rows 2M, contraction 2M) and packed terms (rows n_tot;
// in split-BF16x3 mode padded to that mode's product tile, for V in FP32)
struct TaylorShape {
  long x_rows, y_rows, kchunk, x_wstride, y_wstride;   // strides in floats
};
TaylorShape taylor_shape(afq_system s) {
  TaylorShape t;
  t.x_rows = pad_to(2L * s->M, GeoTY::RB);
  t.y_rows = pad_to(s->ntot, taylor_b3(s) ? 32L * kB3Tiles[b3_tile_of(s)].ta : (long)GeoTY::RA);
  t.kchunk = pad_to(2L * s->M, RK) / RK;
  t.x_wstride = t.x_rows * t.kchunk * RK;
  t.y_wstride = t.y_rows * t.kchunk * RK;
  return t;
}

// the same operands as BF16 hi / lo planes of 32-element chunks (bytes),
// rows padded to the system's product tile
struct TaylorB3Shape {
  long x_rows, y_rows, kchunk, x_plane, x_wstride, y_plane, y_wstride;
  int tile;
};
TaylorB3Shape taylor_b3_shape(afq_system s) {
  TaylorB3Shape t;
  t.tile = b3_tile_of(s);
  t.x_rows = pad_to((long)s->M, 16L * kB3Tiles[t.tile].tb);   // compact rows m of A_w
  t.y_rows = pad_to(s->ntot, 32L * kB3Tiles[t.tile].ta);
  t.kchunk = pad_to(2L * s->M, ring::KC) / ring::KC;
  t.x_plane = t.kchunk * t.x_rows * ROWB;
  t.y_plane = t.kchunk * t.y_rows * ROWB;
  t.x_wstride = 2 * t.x_plane;
  t.y_wstride = 2 * t.y_plane;
  return t;
}
// the B1 products' operands as BF16 hi / lo planes (bytes)
struct B1B3Shape {
  long a_rows, b_rows, kchunk, a_plane, a_wstride, b_plane;
  int tile;
};
B1B3Shape b1_b3_shape(afq_system s) {
  B1B3Shape b;
  b.tile = b3_tile_of(s);
  b.a_rows = pad_to(2L * s->ntot, 32L * kB3Tiles[b.tile].ta);
  b.b_rows = pad_to(s->M, 32L * kB3Tiles[b.tile].tb);
  b.kchunk = pad_to(s->M, ring::KC) / ring::KC;
  b.a_plane = b.kchunk * b.a_rows * ROWB;
  b.a_wstride = 2 * b.a_plane;
  b.b_plane = b.kchunk * b.b_rows * ROWB;
  return b;
}

// walker rows (n, Re|Im) against rows m of B1 - I
struct B1Shape {
  long a_rows, b_rows, kchunk, a_wstride;
};
B1Shape b1_shape(afq_system s) {
  B1Shape b;
  b.a_rows = pad_to(2L * s->ntot, GeoTY::RA);
  b.b_rows = pad_to(s->M, GeoTY::RB);
  b.kchunk = pad_to(s->M, RK) / RK;
  b.a_wstride = b.a_rows * b.kchunk * RK;
  return b;
}

}  // namespace

bool r32_coulomb_used(afq_system s) { return s->lt32[0].p != nullptr; }

// one split-BF16x3 product launch with tile t
template <int MODE>
static int launch_b3(int t, const HornerB3Args& g, hipStream_t st) {
  const long launch = ((long)g.grid + NXCD - 1) / NXCD * NXCD;
  switch (t) {
    case 0: hipLaunchKernelGGL((horner_bf3_kernel<7, 5, MODE>), dim3((unsigned)launch), dim3(256), 0, st, g); break;
    case 1: hipLaunchKernelGGL((horner_bf3_kernel<4, 4, MODE>), dim3((unsigned)launch), dim3(256), 0, st, g); break;
    case 2: hipLaunchKernelGGL((horner_bf3_kernel<2, 2, MODE>), dim3((unsigned)launch), dim3(256), 0, st, g); break;
    default: AFQ_CHECK(false, AFQ_E_INVALID, "split-BF16x3 product: bad tile");
  }
  return hip_status(hipGetLastError(), "split-BF16x3 product");
}

int r32_prepare_b1(afq_system s) {
  if (s->chol32t.p && s->B1.p && taylor_b3(s) && (s->b1x3_dt != s->B1_dt || s->b1x3_tile != b3_tile_of(s))) {
    const B1B3Shape b = b1_b3_shape(s);
    AFQ_RET(s->b1x3.alloc((size_t)2 * b.b_plane));
    hipLaunchKernelGGL(pack_b1_bf3_kernel, dim3(grid_of(b.kchunk * b.b_rows * 32)), dim3(256), 0, s->stream,
                       s->B1.as<double>(), s->M, b.b_rows, (int)b.kchunk, b.b_plane,
                       s->b1x3.as<unsigned short>());
    AFQ_TRY_HIP(hipGetLastError());
    s->b1x3_dt = s->B1_dt;
    s->b1x3_tile = b.tile;
  }
  if (!s->chol32t.p || !s->B1.p || s->b1x_dt == s->B1_dt) return AFQ_OK;
  const B1Shape b = b1_shape(s);
  AFQ_RET(s->b1x.alloc((size_t)b.kchunk * b.b_rows * RK * sizeof(float)));
  hipLaunchKernelGGL(pack_b1_kernel, dim3(grid_of(b.kchunk * b.b_rows * RK)), dim3(256), 0, s->stream,
                     s->B1.as<double>(), s->M, b.b_rows, (int)b.kchunk, s->b1x.as<float>());
  AFQ_TRY_HIP(hipGetLastError());
  s->b1x_dt = s->B1_dt;
  return AFQ_OK;
}

bool r32_b1_packs_terms(afq_system s) { return taylor_b3(s); }

int r32_b1(afq_system s, afq_walkers w, const double2* in, double2* out, hipStream_t st, bool pack_terms,
           bool in_rows_packed) {
  if (taylor_b3(s)) {
    const B1B3Shape b = b1_b3_shape(s);
    AFQ_CHECK(s->b1x3.p && s->b1x3_dt == s->B1_dt && s->b1x3_tile == b.tile && w->r32_layout == 2 + b.tile &&
                  w->r32_b1w.bytes >= (size_t)w->nw * b.a_wstride,
              AFQ_E_STATE, "B1 product (split BF16): operands not prepared");
    if (!in_rows_packed) {   // else the last Horner product wrote them with U
      hipLaunchKernelGGL(pack_walker_rows_bf3_kernel, dim3(ceil_div(s->ntot, 8), (unsigned)b.kchunk, w->nw),
                         dim3(256), 0, st, in, s->M, s->ntot, b.a_rows, b.a_plane, b.a_wstride,
                         w->r32_b1w.as<unsigned char>());
      AFQ_TRY_HIP(hipGetLastError());
    }
    HornerB3Args g{};
    g.a = w->r32_b1w.as<unsigned char>();
    g.b = s->b1x3.as<unsigned char>();
    g.rows_a = b.a_rows;
    g.rows_b = b.b_rows;
    g.a_plane = b.a_plane;
    g.b_plane = b.b_plane;
    g.a_wstride = b.a_wstride;
    g.b_wstride = 0;
    g.nchunk = (int)b.kchunk;
    g.nblk_a = (int)(b.a_rows / (32 * kB3Tiles[b.tile].ta));
    g.nblk_b = (int)(b.b_rows / (32 * kB3Tiles[b.tile].tb));
    g.nw = w->nw;
    const long grid = (long)g.nblk_a * g.nblk_b * w->nw;
    AFQ_CHECK(grid < (1L << 30), AFQ_E_INVALID, "B1 product (split BF16): too many workgroups");
    g.grid = (int)grid;
    g.u = out;
    g.ubase = in;
    g.ntot = s->ntot;
    g.M = s->M;
    if (pack_terms) {   // out is V of the Taylor products: write it in their packed layouts too
      const TaylorShape ts = taylor_shape(s);
      const TaylorB3Shape t3 = taylor_b3_shape(s);
      AFQ_CHECK(w->r32_y[0].bytes >= (size_t)w->nw * ts.y_wstride * sizeof(float) &&
                    w->r32_y[2].bytes >= (size_t)w->nw * t3.y_wstride,
                AFQ_E_STATE, "B1 product (split BF16): term scratch not prepared");
      g.vp = w->r32_y[0].as<float>();
      g.vp_rows = ts.y_rows;
      g.vp_wstride = ts.y_wstride;
      g.vb = w->r32_y[2].as<unsigned char>();
      g.vb_rows = t3.y_rows;
      g.vb_plane = t3.y_plane;
      g.vb_wstride = t3.y_wstride;
    }
    return launch_b3<B3_B1>(b.tile, g, st);
  }
  const B1Shape b = b1_shape(s);
  AFQ_CHECK(s->b1x.p && s->b1x_dt == s->B1_dt && w->r32_b1w.bytes >= (size_t)w->nw * b.a_wstride * sizeof(float),
            AFQ_E_STATE, "B1 product (FP32 ring): operands not prepared");
  hipLaunchKernelGGL(pack_walker_rows_kernel, dim3(ceil_div(s->ntot, 16), ceil_div(s->M, 16), w->nw), dim3(256), 0,
                     st, in, s->M, s->ntot, b.a_rows, b.a_wstride, w->r32_b1w.as<float>());
  AFQ_TRY_HIP(hipGetLastError());
  R32Args g{};
  g.a = w->r32_b1w.as<unsigned char>();
  g.b = s->b1x.as<unsigned char>();
  g.rows_a = b.a_rows;
  g.rows_b = b.b_rows;
  g.a_bstride = b.a_wstride * (long)sizeof(float);
  g.b_bstride = 0;
  g.nchunk = (int)b.kchunk;
  g.kper = (int)b.kchunk;
  g.nbatch = w->nw;
  g.a_fast = 1;
  g.u = out;
  g.ubase = in;
  g.M = s->M;
  g.ntot = s->ntot;
  return launch<GeoTY, EPI_B1>(g, st);
}
bool r32_taylor_used(afq_system s) { return s->chol32t.p != nullptr; }

int r32_prepare(afq_system s) {
  hipStream_t st = s->stream;
  const bool reduced = s->prec != AFQ_FP64 && s->kp_nk == 0;
  if (reduced && !s->chol32t.p) {
    const TriCols tc = tri_cols(s);
    const int nchunk = (int)pad_to(s->X, RK) / RK;
    AFQ_RET(s->tri8.alloc((size_t)tc.nbp * sizeof(int)));
    hipLaunchKernelGGL(tri_table_kernel, dim3(ceil_div(tc.nbp, 256)), dim3(256), 0, st, tc.nb, tc.nbp,
                       s->tri8.as<int>());
    AFQ_TRY_HIP(hipGetLastError());
    AFQ_RET(s->chol32t.alloc((size_t)nchunk * tc.rows * RK * sizeof(float)));
    hipLaunchKernelGGL(pack_tri_cols_kernel, dim3(grid_of((long)nchunk * tc.rows * RK)), dim3(256), 0, st,
                       s->chol.as<double>(), s->M, s->X, s->tri8.as<int>(), tc.ncol, tc.rows, nchunk,
                       s->chol32t.as<float>());
    AFQ_TRY_HIP(hipGetLastError());
  }
  if (reduced && s->prec == AFQ_BF16X3 && !s->chol3.p) {
    const TriCols tc = tri_cols(s);
    const int nchunk = (int)(pad_to(s->X, ring::KC) / ring::KC);
    const long plane = (long)nchunk * tc.rows * ROWB;
    AFQ_RET(s->chol3.alloc((size_t)2 * plane));
    hipLaunchKernelGGL(pack_tri_cols_bf3_kernel, dim3(grid_of((long)nchunk * tc.rows * 32)), dim3(256), 0, st,
                       s->chol.as<double>(), s->M, s->X, s->tri8.as<int>(), tc.ncol, tc.rows, nchunk, plane / 2,
                       s->chol3.as<unsigned short>());
    AFQ_TRY_HIP(hipGetLastError());
  } else if (s->prec != AFQ_BF16X3 && s->chol3.p) {
    s->chol3.free();
  }
  const bool coul = s->prec == AFQ_BF16X3 && s->real_trial && s->kp_nk == 0 && s->msd_n == 0;
  if (coul && !s->lt32[0].p) {
    AFQ_CHECK(s->LtRe.p, AFQ_E_STATE, "force bias (FP32 ring): real half-rotated vectors missing");
    // equal trial blocks give equal half-rotated vectors: one contraction with
    // the spin sum of Theta replaces the two (the assembly only needs the sum)
    bool same = s->n_up == s->n_dn;
    if (same) {
      const int M = s->M, ntot = s->ntot;
      std::vector<double2> ph((size_t)M * ntot);
      AFQ_TRY_HIP(hipMemcpyAsync(ph.data(), s->phi.p, ph.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
      AFQ_TRY_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < M && same; ++i)
        for (int a = 0; a < s->n_up && same; ++a) {
          const double2 x = ph[(size_t)i * ntot + a], y = ph[(size_t)i * ntot + s->n_up + a];
          same = x.x == y.x && x.y == y.y;
        }
    }
    s->lt_share = same;
    for (int sp = 0; sp < (same ? 1 : 2); ++sp) {
      const long NM = (long)s->nspin_n(sp) * s->M;
      const long rows = pad_to(s->X, GeoAB::RB);
      const int nchunk = (int)(pad_to(NM, RK) / RK);
      AFQ_RET(s->lt32[sp].alloc((size_t)nchunk * rows * RK * sizeof(float)));
      hipLaunchKernelGGL(pack_real_rows_kernel, dim3(grid_of((long)nchunk * rows * RK)), dim3(256), 0, st,
                         s->LtRe.as<double>() + (long)s->spin_off(sp) * s->M, (long)s->ntot * s->M, s->X, NM, rows,
                         nchunk, s->lt32[sp].as<float>());
      AFQ_TRY_HIP(hipGetLastError());
    }
  } else if (!coul && s->lt32[0].p) {
    s->lt32[0].free();
    s->lt32[1].free();
    s->lt_share = false;
  }
  if (!reduced && s->chol32t.p) {
    s->chol32t.free();
    s->tri8.free();
  }
  if (!reduced) {
    s->b1x.free();
    s->b1x_dt = -1.0;
  }
  if (s->prec != AFQ_BF16X3) {
    s->b1x3.free();
    s->b1x3_dt = -1.0;
  }
  return r32_prepare_b1(s);
}

// The packed buffers are cleared when allocated: their padding rows and
// contraction columns are never written afterwards and must stay zero (finite).
static int alloc_cleared(DevBuf& b, size_t bytes, hipStream_t st) {
  if (b.bytes >= bytes) return AFQ_OK;
  AFQ_RET(b.alloc(bytes));
  AFQ_TRY_HIP(hipMemsetAsync(b.p, 0, bytes, st));
  return AFQ_OK;
}

int r32_alloc_scratch(afq_system s, afq_walkers w) {
  if (!s->chol32t.p) return AFQ_OK;
  hipStream_t st = s->stream;
  const long rows = coef_rows(w->nw);
  AFQ_RET(alloc_cleared(w->r32_coef, std::max((size_t)pad_to(s->X, RK) * sizeof(float),
                                              (size_t)pad_to(s->X, ring::KC) * 4) * rows, st));
  const TaylorShape ts = taylor_shape(s);
  const TaylorB3Shape t3 = taylor_b3_shape(s);
  const size_t xbytes = std::max((size_t)ts.x_wstride * sizeof(float), (size_t)t3.x_wstride) * w->nw;
  const size_t ybytes = std::max((size_t)ts.y_wstride * sizeof(float), (size_t)t3.y_wstride) * w->nw;
  AFQ_RET(alloc_cleared(w->r32_x, xbytes, st));
  for (int i = 0; i < 3; ++i) AFQ_RET(alloc_cleared(w->r32_y[i], ybytes, st));
  AFQ_RET(alloc_cleared(w->r32_b1w, std::max((size_t)b1_shape(s).a_wstride * sizeof(float),
                                             (size_t)b1_b3_shape(s).a_wstride) * w->nw, st));
  // the FP32 and the BF16 layouts put their zero padding in different places:
  // clear the buffers when the layout changes
  const int layout = taylor_b3(s) ? 2 + b3_tile_of(s) : 1;
  if (w->r32_layout != layout) {
    AFQ_TRY_HIP(hipMemsetAsync(w->r32_x.p, 0, w->r32_x.bytes, st));
    for (int i = 1; i < 3; ++i) AFQ_TRY_HIP(hipMemsetAsync(w->r32_y[i].p, 0, w->r32_y[i].bytes, st));
    AFQ_TRY_HIP(hipMemsetAsync(w->r32_b1w.p, 0, w->r32_b1w.bytes, st));
    AFQ_TRY_HIP(hipMemsetAsync(w->r32_coef.p, 0, w->r32_coef.bytes, st));
    w->r32_layout = layout;
  }

  if (!s->lt32[0].p) return AFQ_OK;
  size_t tb = 0, pb = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const long NM = (long)s->nspin_n(sp) * s->M;
    const long nchunk = pad_to(NM, RK) / RK, rows_b = pad_to(s->X, GeoAB::RB);
    tb = std::max(tb, (size_t)nchunk * rows * RK * sizeof(float));
    const int kper = coulomb_kper(nchunk, rows, rows_b);
    const long nrun = (nchunk + kper - 1) / kper;
    pb = std::max(pb, (size_t)nrun * rows * rows_b * sizeof(float));
  }
  if (w->r32_theta.bytes < tb) AFQ_RET(w->r32_theta.alloc(tb));
  if (w->r32_part.bytes < pb) AFQ_RET(w->r32_part.alloc(pb));
  return AFQ_OK;
}

int r32_abuild(afq_system s, afq_walkers w, const float* coef, hipStream_t st) {
  const long rows = coef_rows(w->nw);
  if (taylor_b3(s)) {   // split BF16 inputs (coefficients and L), A in BF16 planes
    const int nchunk = (int)(pad_to(s->X, ring::KC) / ring::KC);
    const TriCols tc = tri_cols(s);
    const TaylorB3Shape tb = taylor_b3_shape(s);
    const long aplane = (long)nchunk * rows * ROWB, bplane = (long)nchunk * tc.rows * ROWB;
    AFQ_CHECK(s->chol3.p && s->chol3.bytes >= (size_t)2 * bplane && w->r32_layout == 2 + tb.tile &&
                  w->r32_coef.bytes >= (size_t)2 * aplane && w->r32_x.bytes >= (size_t)w->nw * tb.x_wstride,
              AFQ_E_STATE, "propagator build (split BF16): operands not prepared");
    hipLaunchKernelGGL(pack_cplx_rows_bf3_kernel, dim3(grid_of((long)nchunk * rows * 32)), dim3(256), 0, st, coef,
                       (long)s->X, w->nw, (long)s->X, rows, nchunk, aplane / 2, w->r32_coef.as<unsigned short>());
    AFQ_TRY_HIP(hipGetLastError());
    HornerB3Args g{};
    g.a = w->r32_coef.as<unsigned char>();
    g.b = s->chol3.as<unsigned char>();
    g.rows_a = rows;
    g.rows_b = tc.rows;
    g.a_plane = aplane;
    g.b_plane = bplane;
    g.nchunk = nchunk;
    g.nblk_a = (int)(rows / GeoAB::RA);
    g.nblk_b = (int)(tc.rows / GeoAB::RB);
    g.nw = w->nw;
    const long grid = (long)g.nblk_a * g.nblk_b;
    AFQ_CHECK(rows % GeoAB::RA == 0 && tc.rows % GeoAB::RB == 0 && grid < (1L << 30), AFQ_E_INVALID,
              "propagator build (split BF16): bad shape");
    g.grid = (int)grid;
    g.M = s->M;
    g.tri = s->tri8.as<int>();
    g.x = w->r32_x.as<unsigned char>();
    g.x_rows = tb.x_rows;
    g.x_plane = tb.x_plane;
    g.x_wstride = tb.x_wstride;
    g.ncol = tc.ncol;
    const long launch = (grid + NXCD - 1) / NXCD * NXCD;
    hipLaunchKernelGGL((horner_bf3_kernel<GeoAB::TA, GeoAB::TB, B3_XFORM>), dim3((unsigned)launch), dim3(256), 0, st,
                       g);
    return hip_status(hipGetLastError(), "propagator build (split BF16)");
  }
  const int nchunk = (int)(pad_to(s->X, RK) / RK);
  const TaylorShape ts = taylor_shape(s);
  AFQ_CHECK(s->chol32t.p && w->r32_coef.bytes >= (size_t)nchunk * rows * RK * sizeof(float) &&
                w->r32_x.bytes >= (size_t)w->nw * ts.x_wstride * sizeof(float),
            AFQ_E_STATE, "propagator build (FP32 ring): operands not prepared");
  hipLaunchKernelGGL(pack_cplx_rows_kernel<float>, dim3(grid_of((long)nchunk * rows * RK)), dim3(256), 0, st, coef,
                     (long)s->X, w->nw, (long)s->X, rows, nchunk, w->r32_coef.as<float>());
  AFQ_TRY_HIP(hipGetLastError());
  R32Args g{};
  g.a = w->r32_coef.as<unsigned char>();
  g.b = s->chol32t.as<unsigned char>();
  g.rows_a = rows;
  const TriCols tc = tri_cols(s);
  g.rows_b = tc.rows;
  g.nchunk = nchunk;
  g.kper = nchunk;
  g.a_fast = 1;
  g.tri = s->tri8.as<int>();
  g.x = w->r32_x.as<float>();
  g.x_wstride = ts.x_wstride;
  g.x_rows = ts.x_rows;
  g.ncol = tc.ncol;
  g.M = s->M;
  g.nw = w->nw;
  return launch<GeoAB, EPI_XFORM>(g, st);
}

// U <- T_K(A) U in Horner form with split-BF16x3 products
static int r32_taylor_b3(afq_system s, afq_walkers w, int order, hipStream_t st, bool terms_packed,
                         bool* b1_rows) {
  const TaylorShape ts = taylor_shape(s);
  const TaylorB3Shape tb = taylor_b3_shape(s);
  AFQ_CHECK(w->r32_layout == 2 + tb.tile && w->r32_x.bytes >= (size_t)w->nw * tb.x_wstride &&
                w->r32_y[0].bytes >= (size_t)w->nw * ts.y_wstride * sizeof(float) &&
                w->r32_y[1].bytes >= (size_t)w->nw * tb.y_wstride && w->r32_y[2].bytes >= (size_t)w->nw * tb.y_wstride,
            AFQ_E_STATE, "Taylor propagator (split BF16): walker scratch not prepared");
  const B3Tile tl = kB3Tiles[tb.tile];
  AFQ_CHECK(ts.y_rows == tb.y_rows && tb.y_rows % (32 * tl.ta) == 0 && tb.x_rows % (16 * tl.tb) == 0, AFQ_E_INVALID,
            "Taylor propagator (split BF16): bad shape");
  if (order < 1) return AFQ_OK;
  // V in FP32 (added by every epilogue) and as BF16 planes (the first input),
  // unless the B1 product that formed V wrote them
  if (!terms_packed) {
    hipLaunchKernelGGL(pack_terms_kernel, dim3(ceil_div(s->ntot, 32), ceil_div(s->M, 8), w->nw), dim3(256), 0, st,
                       w->u.as<double2>(), s->M, s->ntot, ts.y_rows, ts.y_wstride, w->r32_y[0].as<float>());
    AFQ_TRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(pack_terms_bf3_kernel, dim3(ceil_div(s->ntot, 16), ceil_div(s->M, 16), w->nw), dim3(256), 0,
                       st, w->u.as<double2>(), s->M, s->ntot, tb.y_rows, tb.y_plane, tb.y_wstride,
                       w->r32_y[2].as<unsigned char>());
    AFQ_TRY_HIP(hipGetLastError());
  }
  HornerB3Args g{};
  g.b = w->r32_x.as<unsigned char>();
  g.rows_a = tb.y_rows;
  g.rows_b = tb.x_rows;
  g.a_plane = tb.y_plane;
  g.b_plane = tb.x_plane;
  g.a_wstride = tb.y_wstride;
  g.b_wstride = tb.x_wstride;
  g.nchunk = (int)tb.kchunk;
  g.nblk_a = (int)(tb.y_rows / (32 * tl.ta));
  g.nblk_b = (int)(tb.x_rows / (16 * tl.tb));
  g.nw = w->nw;
  const long grid = (long)g.nblk_a * g.nblk_b * w->nw;
  AFQ_CHECK(grid < (1L << 30), AFQ_E_INVALID, "Taylor propagator (split BF16): too many workgroups");
  g.grid = (int)grid;
  g.vy = w->r32_y[0].as<float>();
  g.vy_rows = ts.y_rows;
  g.vy_wstride = ts.y_wstride;
  g.u = w->u.as<double2>();
  g.ntot = s->ntot;
  g.M = s->M;
  const unsigned char* in = w->r32_y[2].as<unsigned char>();
  for (int j = order; j >= 1; --j) {
    unsigned char* out = w->r32_y[1 + (order - j) % 2].as<unsigned char>();
    g.a = in;
    g.yout = out;
    g.scale = 1.0f / (float)j;
    if (j == 1) {
      if (b1_rows) {   // U also as the walker rows of the B1 product that follows
        const B1B3Shape b = b1_b3_shape(s);
        AFQ_CHECK(w->r32_b1w.bytes >= (size_t)w->nw * b.a_wstride, AFQ_E_STATE,
                  "Taylor propagator (split BF16): B1 walker rows not prepared");
        g.wr = w->r32_b1w.as<unsigned char>();
        g.wr_rows = b.a_rows;
        g.wr_plane = b.a_plane;
        g.wr_wstride = b.a_wstride;
        *b1_rows = true;
      }
      AFQ_RET(launch_b3<B3_HORNER_LAST>(tb.tile, g, st));
    } else {
      AFQ_RET(launch_b3<B3_HORNER>(tb.tile, g, st));
    }
    in = out;
  }
  return AFQ_OK;
}

int r32_taylor(afq_system s, afq_walkers w, int order, hipStream_t st, bool terms_packed, bool* b1_rows) {
  if (b1_rows) *b1_rows = false;
  if (taylor_b3(s)) return r32_taylor_b3(s, w, order, st, terms_packed, b1_rows);
  const TaylorShape ts = taylor_shape(s);
  const size_t yb = (size_t)w->nw * ts.y_wstride * sizeof(float);
  AFQ_CHECK(w->r32_x.bytes >= (size_t)w->nw * ts.x_wstride * sizeof(float) && w->r32_y[0].bytes >= yb &&
                w->r32_y[1].bytes >= yb && w->r32_y[2].bytes >= yb,
            AFQ_E_STATE, "Taylor propagator (FP32 ring): walker scratch not prepared");
  if (order < 1) return AFQ_OK;
  float* V = w->r32_y[0].as<float>();
  hipLaunchKernelGGL(pack_terms_kernel, dim3(ceil_div(s->ntot, 32), ceil_div(s->M, 8), w->nw), dim3(256), 0, st,
                     w->u.as<double2>(), s->M, s->ntot, ts.y_rows, ts.y_wstride, V);
  AFQ_TRY_HIP(hipGetLastError());
  const float* in = V;
  for (int j = order; j >= 1; --j) {
    float* out = w->r32_y[1 + (order - j) % 2].as<float>();
    R32Args g{};
    g.a = reinterpret_cast<const unsigned char*>(in);
    g.b = w->r32_x.as<unsigned char>();
    g.rows_a = ts.y_rows;
    g.rows_b = ts.x_rows;
    g.a_bstride = ts.y_wstride * (long)sizeof(float);
    g.b_bstride = ts.x_wstride * (long)sizeof(float);
    g.nchunk = (int)ts.kchunk;
    g.kper = (int)ts.kchunk;
    g.nbatch = w->nw;
    g.a_fast = 0;
    g.vy = V;
    g.yout = out;
    g.u = w->u.as<double2>();
    g.scale = 1.0f / (float)j;
    g.y_rows = ts.y_rows;
    g.y_wstride = ts.y_wstride;
    g.ntot = s->ntot;
    g.M = s->M;
    if (j == 1) AFQ_RET((launch<GeoTY, EPI_HORNER_LAST>(g, st)));
    else AFQ_RET((launch<GeoTY, EPI_HORNER>(g, st)));
    in = out;
  }
  return AFQ_OK;
}

int r32_coulomb(afq_system s, afq_walkers w, hipStream_t st) {
  AFQ_CHECK(s->lt32[0].p && (s->lt_share || s->lt32[1].p), AFQ_E_STATE,
            "force bias (FP32 ring): operands not prepared");
  const long rows = coef_rows(w->nw), rows_b = pad_to(s->X, GeoAB::RB);
  const bool both = s->lt_share;   // one contraction of the spin sum (equal trial blocks)
  for (int sp = 0; sp < (both ? 1 : 2); ++sp) {
    const long NM = (long)s->nspin_n(sp) * s->M;
    const int nchunk = (int)(pad_to(NM, RK) / RK);
    const int kper = coulomb_kper(nchunk, rows, rows_b);
    const int nrun = (nchunk + kper - 1) / kper;
    AFQ_CHECK(w->r32_theta.bytes >= (size_t)nchunk * rows * RK * sizeof(float) &&
                  w->r32_part.bytes >= (size_t)nrun * rows * rows_b * sizeof(float),
              AFQ_E_STATE, "force bias (FP32 ring): walker scratch not prepared");
    // Theta-hat rows (w, Re|Im): thetaT[w][off + a][k] at (a, k) -> a M + k
    // (with both: thetaT[w][a][k] + thetaT[w][n_up + a][k])
    const double* th = reinterpret_cast<const double*>(w->theta.as<double2>() + (long)s->spin_off(sp) * s->M);
    if (both)
      hipLaunchKernelGGL(pack_cplx_rows_sum_kernel, dim3(grid_of((long)nchunk * rows * RK)), dim3(256), 0, st, th,
                         (long)s->ntot * s->M, (long)s->spin_off(1) * s->M, w->nw, NM, rows, nchunk,
                         w->r32_theta.as<float>());
    else
      hipLaunchKernelGGL(pack_cplx_rows_kernel<double>, dim3(grid_of((long)nchunk * rows * RK)), dim3(256), 0, st,
                         th, (long)s->ntot * s->M, w->nw, NM, rows, nchunk, w->r32_theta.as<float>());
    AFQ_TRY_HIP(hipGetLastError());
    R32Args g{};
    g.a = w->r32_theta.as<unsigned char>();
    g.b = s->lt32[sp].as<unsigned char>();
    g.rows_a = rows;
    g.rows_b = rows_b;
    g.nchunk = nchunk;
    g.kper = kper;
    g.a_fast = 0;
    g.part = w->r32_part.as<float>();
    AFQ_RET((launch<GeoAB, EPI_PART>(g, st)));
    hipLaunchKernelGGL(coulomb_reduce_kernel, dim3(grid_of((long)w->nw * s->X)), dim3(256), 0, st,
                       w->r32_part.as<float>(), nrun, rows, rows_b, w->nw, s->X, sp, both ? 1 : 0,
                       w->tro.as<double2>());
    AFQ_TRY_HIP(hipGetLastError());
  }
  return AFQ_OK;
}

// Pins the split-BF16x3 product tile (-1: the padded-work model) and repacks
// B1 - I for it; walker sets clear their packed operands for the new layout
// at their next call, and captured batches capture again (version).
int system_set_b3_tile(afq_system s, int tile) {
  AFQ_CHECK(tile >= -1 && tile < kNumB3Tiles, AFQ_E_INVALID, "propagator tile must be -1.." + std::to_string(kNumB3Tiles - 1));
  if (s->b3_tile == tile) return AFQ_OK;
  s->b3_tile = tile;
  if (s->B1.p) AFQ_RET(r32_prepare_b1(s));
  AFQ_TRY_HIP(hipStreamSynchronize(s->stream));
  ++s->version;
  return AFQ_OK;
}

// Times one step's split-BF16x3 products (the first B1 product, which packs
// the Taylor terms, and the order-6 Horner chain; the second B1 product is
// the first's kind) with every tile on these walkers' own shapes, `reps`
// times each with HIP events, and pins the fastest. Writes only per-step
// scratch (U, the packed terms and operands); W is read.
int r32_autotune(afq_system s, afq_walkers w, int reps, int* tile_out) {
  *tile_out = -1;
  if (!taylor_b3(s) || !s->chol32t.p || s->kp_nk > 0) return AFQ_OK;   // the ring products are not in use
  hipStream_t st = s->stream;
  if (!s->B1.p) AFQ_RET(system_prepare_dt(s, 0.01));   // any step size: only the timing matters
  hipEvent_t e0 = nullptr, e1 = nullptr;
  AFQ_TRY_HIP(hipEventCreate(&e0));
  AFQ_TRY_HIP(hipEventCreate(&e1));
  int rc = AFQ_OK, best = -1;
  float best_ms = 0.f;
  const int pinned = s->b3_tile;
  for (int t = 0; t < kNumB3Tiles && rc == AFQ_OK; ++t) {
    if ((rc = system_set_b3_tile(s, t)) != AFQ_OK) break;
    if ((rc = walkers_alloc_scratch(w)) != AFQ_OK) break;
    if ((rc = hip_status(hipEventRecord(e0, st), "hipEventRecord")) != AFQ_OK) break;
    for (int r = 0; r < reps && rc == AFQ_OK; ++r) {
      rc = r32_b1(s, w, w->W.as<double2>(), w->u.as<double2>(), st, true);
      if (rc == AFQ_OK) rc = r32_taylor(s, w, 6, st, true);
    }
    if (rc != AFQ_OK) break;
    if ((rc = hip_status(hipEventRecord(e1, st), "hipEventRecord")) != AFQ_OK) break;
    if ((rc = hip_status(hipEventSynchronize(e1), "hipEventSynchronize")) != AFQ_OK) break;
    float ms = 0.f;
    if ((rc = hip_status(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) != AFQ_OK) break;
    if (best < 0 || ms < best_ms) {
      best = t;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != AFQ_OK) {
    (void)system_set_b3_tile(s, pinned);
    (void)walkers_alloc_scratch(w);
    return rc;
  }
  AFQ_RET(system_set_b3_tile(s, best));
  AFQ_RET(walkers_alloc_scratch(w));
  *tile_out = best;
  return AFQ_OK;
}

