// Exchange through the half-rotated four-index tensor (split-BF16x3 and FP64
// modes, real trial). With Theta-hat = vec(Theta^s), index (a, k) -> a M + k,
// the sum over Cholesky vectors of tr(Omega_n Omega_n) is one quadratic form,
//   sum_n tr(Omega_n Omega_n) = Theta-hat^T W' Theta-hat,
//   W'[(b,k),(a,l)] = sum_n Lt_n[a][k] Lt_n[b][l]      (Lt_n = T^H L^n, N x M),
// W' symmetric of order N M. Cut into blocks of RA rows, the form is
//   sum_p theta_p^T W'_pp theta_p + 2 sum_{p<q} theta_p^T W'_pq theta_q,
// so only the upper block triangle is stored and contracted: W'' = W' on the
// diagonal blocks, 2 W' above them (exact in BF16), and row block p runs over
// the contraction columns from its own diagonal block on. Per walker and spin
// that is (N M)^2 / 2 multiply-adds instead of the X N^2 M of the Cholesky
// form (1/8 of it at M = 400, X = 1600), for about (N M)^2 / 2 stored entries
// (BF16 hi and lo planes: 3.2 GB per distinct spin block at M = 400, N = 100).
//
// W' is formed once per system, one column slab a (columns (a, l), l < M) at
// a time: with LT[(a,k)][n] = Lt_n[a][k], the FP64 GEMM LT_a LT^T over n gives
// W[(a,k)][(b,l)] = W'[(b,k)][(a,l)] for the rows the triangle keeps, and a
// pack kernel permutes, weights and splits them into the stored layout (the
// transients are LT and one M x N M slab, not the whole N M x N M matrix).
// Per step: Theta-hat of every walker is packed into rows (w, Re|Im); the
// kernel multiplies W'' (rows I) by Theta-hat (rows C) in split BF16x3 through
// the three-stage direct global->LDS ring, one work unit being a row block and
// a contiguous run of contraction chunks; its epilogue contracts the FP32 tile
// with Theta-hat in FP64 (no output matrix is stored) and writes one complex
// partial per (unit, column); a fixed-order reduction gives every walker's sum.
//
// FP64 mode keeps W' itself, its columns cut into NB blocks J and block column
// J stored down to the end of its diagonal block ((1/2 + 1/(2 NB)) of the
// square, 7.2 GB at M = 400), and runs the same quadratic form on FP64 MFMA
// through the tiled GEMM: Z_J^T = 2 Theta-hat_{<J}^T W'_{<J,J} +
// Theta-hat_J^T W'_JJ (two GEMMs per block), then one FP64 dot product per
// walker, sum_I Theta-hat_I Z_I.
#include <algorithm>
#include <cmath>
#include <vector>
#include "mfma_ring.h"
#include "common.h"
#include "step_kernels.h"

namespace {

using ring::bf16x8;
using ring::dma16s;
using ring::f4;
using ring::KC;
using ring::lds_t;
using ring::ROWB;
using ring::swz;
using ring::wait_vm_barrier;

constexpr int NWAVE = 4;
constexpr int TA = 8, TB = 4;               // 16 x 16 tiles per wave: W'' rows x Theta-hat rows
constexpr int RA = 32 * TA, RBR = 32 * TB;  // workgroup tile: 256 x 128 (2 x 2 waves)
constexpr int REGA = RA * ROWB, REGB = RBR * ROWB;
constexpr int STAGE = 2 * REGA + 2 * REGB;  // A hi, A lo, B hi, B lo
constexpr int NT = STAGE / 1024;            // 1 KB load instructions per stage
constexpr int NQ = NT / NWAVE;              // per wave
static_assert(NT % NWAVE == 0, "loads must split evenly over the waves");
constexpr int NXCD = 8;
constexpr int CPB = RA / KC;                // contraction chunks per row block
// the loads of the A regions (W'' hi, lo) are the first QA of every wave's NQ
constexpr int QA = (RA / 8) / NWAVE;
static_assert((RA / 8) % NWAVE == 0, "every wave's loads must split into A and B regions at the same index");

// Upper block triangle of W'' in chunk-major planes: chunk c (columns
// [KC c, KC c + KC)) stores the rows of the row blocks 0 .. c / CPB, whose
// diagonal block it reaches, after the rows of all earlier chunks
__host__ __device__ inline long tri_rows(long c) { return (c / CPB + 1) * RA; }
__host__ __device__ inline long tri_rows_before(long c) {
  const long q = c / CPB, r = c - q * CPB;
  return RA * (CPB * q * (q + 1) / 2 + r * (q + 1));
}

struct EriArgs {
  const unsigned char* a[2];   // W'' hi / lo planes: chunk c at row tri_rows_before(c), 32 bf16 per row
  const unsigned char* b[2];   // Theta-hat hi / lo planes: [chunk][rows_b][32] bf16
  long rows_b;
  const int4* units;           // (row block, first chunk, chunks, interval)
  const int2* wg;              // (unit, column block) of workgroup i, unit < 0: idle
  const double2* thetaT;       // nw x ntot x M
  int ntot, M, off, NM, nw;
  int off1, nsp;               // column walkers nsp * nw: walker w of spin 1 (offset off1) at nw + w
  double2* part;               // [unit][rows_b]
};

// the wave-uniform base of load q of chunk ch of a work unit (chunk c0 + ch
// of the run): W'' chunks start at their triangle row offset, Theta-hat
// chunks rows_b rows apart; qb[q] is the load's first row in chunk 0
struct EriLoader {
  const unsigned char* qb[NQ];
  long bstride;
  int c0;
  __device__ const unsigned char* src(int q, int ch) const {
    return qb[q] + (q < QA ? tri_rows_before(c0 + ch) * ROWB : (long)(c0 + ch) * bstride);
  }
};

__global__ __launch_bounds__(256, 1) void eri_kernel(EriArgs g) {
  __shared__ __align__(16) unsigned char L0[STAGE];
  __shared__ __align__(16) unsigned char L1[STAGE];
  __shared__ __align__(16) unsigned char L2[STAGE];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: scalar address arithmetic
  const int rb = wave >> 1, cb = wave & 1;        // row half (W''), column half (Theta-hat)
  // the launch layout (host-built, XCD-aware) names this workgroup's unit
  // and column block
  const int2 e = g.wg[blockIdx.x];
  if (e.x < 0) return;
  const int u = e.x, bb = e.y;
  const int4 un = g.units[u];
  const int c0 = un.y, nc = un.z;                 // nc >= 1
  const long arow0 = (long)un.x * RA, brow0 = (long)bb * RBR;
  // load q of this wave: instruction t = q * 4 + wave of the stage, 16 rows of
  // one region (A hi, A lo, B hi, B lo) starting at row 16 j of the region
  EriLoader ld;
  ld.bstride = g.rows_b * ROWB;
  ld.c0 = c0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int t = q * NWAVE + wave;
    const int reg = t < RA / 16 ? 0 : t < RA / 8 ? 1 : t < RA / 8 + RBR / 16 ? 2 : 3;
    const int j = reg == 0 ? t : reg == 1 ? t - RA / 16 : reg == 2 ? t - RA / 8 : t - RA / 8 - RBR / 16;
    const unsigned char* base = reg == 0 ? g.a[0] : reg == 1 ? g.a[1] : reg == 2 ? g.b[0] : g.b[1];
    ld.qb[q] = base + ((q < QA ? arow0 : brow0) + 16 * j) * ROWB;
  }
  f4 acc[TA][TB];
#pragma unroll
  for (int i = 0; i < TA; ++i)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int arow = rb * (RA / 2), brow = cb * (RBR / 2);
  ring::bf3_stream<TA, TB, REGA, REGB, NQ>(acc, (const lds_t*)L0, (const lds_t*)L1, (const lds_t*)L2,
                                           nc, arow, brow, lane, wave, ld);
  __syncthreads();
  const int lr = lane & 15, lq = lane >> 4;

  // epilogue: column C = (w, part) holds Re (part 0) or Im (part 1) of
  // (W'' Theta-hat_w) over this unit's chunks; its share of the complex form
  // Theta-hat_w . (W'' Theta-hat_w) is theta Z (part 0) or i theta Z (part 1),
  // with the products in FP64
  double sre[TB], sim[TB];
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    sre[j] = sim[j] = 0.0;
    const long C = brow0 + brow + 16 * j + lr;
    const int wc = (int)(C >> 1), pt = (int)(C & 1);
    const bool okc = wc < g.nsp * g.nw;
    const bool s1 = wc >= g.nw;
    const int wk = okc ? wc - (s1 ? g.nw : 0) : 0;
    const double2* th = g.thetaT + ((long)wk * g.ntot + (s1 ? g.off1 : g.off)) * g.M;
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long I = arow0 + arow + 16 * i + 4 * lq + r;
        const bool ok = okc && I < g.NM;
        const double2 tv = th[ok ? I : 0];
        const double z = ok ? (double)acc[i][j][r] : 0.0;
        sre[j] += z * (pt ? -tv.y : tv.x);
        sim[j] += z * (pt ? tv.x : tv.y);
      }
  }
#pragma unroll
  for (int j = 0; j < TB; ++j)
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
      sre[j] += __shfl_xor(sre[j], o);
      sim[j] += __shfl_xor(sim[j], o);
    }
  double* red = reinterpret_cast<double*>(L0);   // [cb][j][lr][2] from the rb = 1 waves
  if (rb == 1 && lane < 16)
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      red[((cb * TB + j) * 16 + lane) * 2] = sre[j];
      red[((cb * TB + j) * 16 + lane) * 2 + 1] = sim[j];
    }
  __syncthreads();
  if (rb == 0 && lane < 16) {
    double2* out = g.part + (long)u * g.rows_b;
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      const long C = brow0 + brow + 16 * j + lane;
      out[C] = make_double2(sre[j] + red[((cb * TB + j) * 16 + lane) * 2],
                            sim[j] + red[((cb * TB + j) * 16 + lane) * 2 + 1]);
    }
  }
}

// split BF16: x -> f = fp32(x); hi = bf16(f); lo = bf16(f - hi), both rounded to nearest even
__device__ inline unsigned short bf16_rne(float f) {
  const unsigned u = __float_as_uint(f);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Column slab a of W'' into the triangle planes. C[k][b M + l] =
// W[(a,k)][(b,l)] = W'[(b,k)][(a,l)] for the rows b M + k < n_rows of the slab
// GEMM. Chunks c_first .. c_first + ncs - 1 overlap the slab; the slab writes
// the columns J = a M + l it owns (the last slab also the zero columns
// J >= NM) of every stored row I < tri_rows(c): W'' = s W', s = 1 on the
// diagonal block (I / RA = J / RA) and 2 above it, zero in the rows I >= NM.
// One thread per element, consecutive threads along a row (contiguous reads
// of C and writes of the planes).
__global__ void eri_pack_slab_kernel(const double* __restrict__ C, long ldc, int M, long NM, int a, long c_first,
                                     int ncs, long rmax, int last, unsigned short* __restrict__ hi,
                                     unsigned short* __restrict__ lo) {
  const long total = (long)ncs * rmax * KC, j_lo = (long)a * M, j_hi = j_lo + M;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long ci = e / (rmax * KC), rem = e - ci * rmax * KC;
    const long I = rem / KC, jj = rem - I * KC, c = c_first + ci, J = c * KC + jj;
    if (I >= tri_rows(c) || J < j_lo || (J >= j_hi && !(last && J >= NM))) continue;
    float f = 0.f;
    if (I < NM && J < NM) {
      const long b = I / M, k = I - b * M, l = J - j_lo;
      const double v = C[k * ldc + b * M + l];
      f = (float)(I / RA == J / RA ? v : 2.0 * v);
    }
    const long o = tri_rows_before(c) * KC + I * KC + jj;
    const unsigned short h = bf16_rne(f);
    hi[o] = h;
    lo[o] = bf16_rne(f - bf16_f(h));
  }
}

// Column slab a of W' into the FP64 block columns: column J = a M + l belongs
// to block Jb = J / bw (columns [j0, j0 + nj)), stored row-major with ld
// f64_ld(nj) down to row j0 + nj (the blocks above the diagonal and the
// diagonal block) at f64_base(Jb); C as for eri_pack_slab_kernel
__host__ __device__ inline long f64_ld(long nj) { return (nj + 1) / 2 * 2; }
__host__ __device__ inline long f64_base(long Jb, long bw) { return bw * bw * Jb * (Jb + 1) / 2; }
__global__ void eri_pack_slab_f64_kernel(const double* __restrict__ C, long ldc, int M, long NM, int a, long bw,
                                         long rmax, double* __restrict__ out) {
  const long total = rmax * M;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long I = e / M, l = e - I * M, J = (long)a * M + l;
    const long Jb = J / bw, j0 = Jb * bw, nj = NM - j0 < bw ? NM - j0 : bw;
    if (I >= j0 + nj) continue;
    const long b = I / M, k = I - b * M;
    out[f64_base(Jb, bw) + I * f64_ld(nj) + (J - j0)] = C[k * ldc + b * M + l];
  }
}

// Theta-hat rows C = 2 w + part of one spin into chunk-major hi / lo planes:
// one thread per (chunk, walker, element of the chunk), both parts
// (nsp = 2: walker w of spin 1, at offset off1, is column walker nw + w)
__global__ void eri_pack_theta_kernel(const double2* __restrict__ thetaT, int ntot, int M, int off, int off1, int nsp,
                                      int NM, int nw, long rows_b, int nchunk, unsigned short* __restrict__ hi,
                                      unsigned short* __restrict__ lo) {
  const long hw = rows_b / 2;
  const long total = (long)nchunk * hw * KC;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long c = e / (hw * KC), rem = e - c * hw * KC;
    const long wk = rem / KC, jj = rem - wk * KC, J = c * KC + jj;
    double2 v = make_double2(0.0, 0.0);
    if (wk < (long)nsp * nw && J < NM) {
      const bool s1 = wk >= nw;
      v = thetaT[((wk - (s1 ? nw : 0)) * ntot + (s1 ? off1 : off)) * M + J];
    }
    const long o = (c * rows_b + 2 * wk) * KC + jj;
    const float fr = (float)v.x, fi = (float)v.y;
    const unsigned short hr = bf16_rne(fr), him = bf16_rne(fi);
    hi[o] = hr;
    hi[o + KC] = him;
    lo[o] = bf16_rne(fr - bf16_f(hr));
    lo[o + KC] = bf16_rne(fi - bf16_f(him));
  }
}

// per walker (one 256-thread workgroup): the sum over units and both parts ->
// troo[w][spin][0], thread t taking units t, t + 256, ... and a fixed-shape tree
// combining the threads (the same order on every call); the other vectors'
// entries are zero (the assembly only sums them)
__global__ __launch_bounds__(256) void eri_reduce_kernel(const double2* __restrict__ part, int nunit, long rows_b,
                                                         int nw, int spin, int X, double2* __restrict__ troo) {
  __shared__ double2 red[256];
  const int w = blockIdx.x, t = threadIdx.x;
  double2 s = make_double2(0.0, 0.0);
  for (int u = t; u < nunit; u += 256) {
    const double2* p = part + (long)u * rows_b + 2L * w;
    s = cadd(s, cadd(p[0], p[1]));
  }
  red[t] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] = cadd(red[t], red[t + h]);
    __syncthreads();
  }
  double2* o = troo + ((long)w * 2 + spin) * X;
  if (t == 0) o[0] = red[0];
  for (int n = 1 + t; n < X; n += 256) o[n] = make_double2(0.0, 0.0);
}

// out[c][r] = in[r * ld_in + c]  (rows x cols -> cols x rows)
__global__ void transpose_real_kernel(const double* __restrict__ in, long rows, long cols, long ld_in,
                                      double* __restrict__ out) {
  const long total = rows * cols;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long c = e / rows, r = e - c * rows;
    out[e] = in[r * ld_in + c];
  }
}

int grid_of(long total) { return (int)std::min<long>(std::max<long>((total + 255) / 256, 1), 1 << 20); }

struct Shape {
  long NM, rows_a;
  int nchunk, nblk_a;
};
Shape shape_of(afq_system s, int sp) {
  Shape h;
  h.NM = (long)s->nspin_n(sp) * s->M;
  h.rows_a = (h.NM + RA - 1) / RA * RA;
  h.nchunk = (int)((h.NM + KC - 1) / KC);
  h.nblk_a = (int)(h.rows_a / RA);
  return h;
}
size_t plane_bytes(long rows, int nchunk) { return (size_t)rows * nchunk * KC * 2; }
// one plane of the W'' triangle
size_t plane_a_bytes(const Shape& h) { return (size_t)tri_rows_before(h.nchunk) * ROWB; }
long rows_b_of(int nw) { return (2L * nw + RBR - 1) / RBR * RBR; }

// work units: row block p covers chunks [CPB p, nchunk), cut at the multiples
// of the interval length R, so that the units of different row blocks in one
// interval cover the same chunks (their Theta-hat chunks are then shared by
// the workgroups resident together on an XCD); unit = (p, first chunk,
// chunks, interval)
std::vector<int> make_units(const Shape& h, int R) {
  std::vector<int> u;
  for (int k = 0; (long)k * R < h.nchunk; ++k)
    for (int p = 0; p < h.nblk_a; ++p) {
      const long lo = std::max((long)k * R, (long)CPB * p), hi = std::min((long)(k + 1) * R, (long)h.nchunk);
      if (lo >= hi) continue;
      u.push_back(p);
      u.push_back((int)lo);
      u.push_back((int)(hi - lo));
      u.push_back(k);
    }
  return u;
}

// interval length: the longer the runs, the fewer workgroups pay the fixed
// cost of the prologue, epilogue and partial sums (at M = 400 whole rows ran
// 5% faster than runs of 256 chunks and 2% faster than 512). With at least
// 128 row blocks whole rows fill the device (times the walkers' column
// blocks); fewer row blocks are cut into about 256 runs of at least 16 chunks.
int choose_interval(const Shape& h) {
  if (h.nblk_a >= 128) return h.nchunk;
  long total = 0;
  for (int p = 0; p < h.nblk_a; ++p) total += h.nchunk - (long)CPB * p;
  return (int)std::min<long>(h.nchunk, std::max<long>(16, (total + 255) / 256));
}

// Launch layout: tiles of G row blocks x CBG column blocks (about one XCD's
// 32 workgroups at one per CU) on one interval, so that each W'' chunk is read
// by the CBG workgroups of its row block and each Theta-hat chunk by the G
// row blocks, all resident on one XCD at the same time and sharing its L2.
// Tiles are dealt to the XCDs longest first, each to the least loaded one
// (work: chunks plus a fixed cost per workgroup), and laid out so that
// workgroup i runs on XCD i % 8 (the hardware's round-robin) in that order.
// Returns (unit, column block) pairs, (-1, -1) for the idle padding.
std::vector<int> make_wg_layout(const std::vector<int>& units, int nblk_a, int nblk_b) {
  constexpr long kOverhead = 6;   // fixed cost of a workgroup, in chunks
  const int CBG = std::min(nblk_b, 8), G = std::max(1, 32 / CBG);
  const int nu = (int)(units.size() / 4);
  int nk = 0;
  for (int i = 0; i < nu; ++i) nk = std::max(nk, units[4 * i + 3] + 1);
  std::vector<int> at((size_t)nk * nblk_a, -1);   // unit of (interval, row block)
  for (int i = 0; i < nu; ++i) at[(size_t)units[4 * i + 3] * nblk_a + units[4 * i]] = i;
  struct Tile { long work; std::vector<int> wg; };
  std::vector<Tile> tiles;
  for (int k = 0; k < nk; ++k)
    for (int p0 = 0; p0 < nblk_a; p0 += G)
      for (int b0 = 0; b0 < nblk_b; b0 += CBG) {
        Tile t{0, {}};
        for (int p = p0; p < std::min(p0 + G, nblk_a); ++p) {
          const int u = at[(size_t)k * nblk_a + p];
          if (u < 0) continue;
          for (int b = b0; b < std::min(b0 + CBG, nblk_b); ++b) {
            t.wg.push_back(u);
            t.wg.push_back(b);
            t.work += units[4 * u + 2] + kOverhead;
          }
        }
        if (!t.wg.empty()) tiles.push_back(std::move(t));
      }
  std::stable_sort(tiles.begin(), tiles.end(), [](const Tile& a, const Tile& b) { return a.work > b.work; });
  std::vector<std::vector<int>> per(NXCD);
  long load[NXCD] = {};
  for (const Tile& t : tiles) {
    const int x = (int)(std::min_element(load, load + NXCD) - load);
    load[x] += t.work;
    per[x].insert(per[x].end(), t.wg.begin(), t.wg.end());
  }
  size_t len = 0;
  for (auto& v : per) len = std::max(len, v.size() / 2);
  std::vector<int> out(2 * NXCD * len, -1);
  for (int x = 0; x < NXCD; ++x)
    for (size_t i = 0; i < per[x].size() / 2; ++i) {
      out[2 * (i * NXCD + x)] = per[x][2 * i];
      out[2 * (i * NXCD + x) + 1] = per[x][2 * i + 1];
    }
  return out;
}

void eri_free(afq_system s) {
  for (int sp = 0; sp < 2; ++sp) {
    s->eri_w[sp].free();
    s->eri_units[sp].free();
    s->eri_nunit[sp] = 0;
    s->eri_units_host[sp].clear();
  }
  s->eri_ready = false;
  s->eri_prec = -1;
}

// column blocks of the FP64 form: NB about 8, widths a multiple of 32 (16-byte
// aligned column offsets for the tiled GEMM)
constexpr int NB64 = 8;
long blk64(long NM) { return std::max<long>(32, (NM + NB64 - 1) / NB64 + 31) / 32 * 32; }

// bytes of the stored tensor of one distinct spin block in the given precision
size_t tensor_bytes_of(const Shape& h, int prec) {
  if (prec != AFQ_FP64) return 2 * plane_a_bytes(h);
  const long bw = blk64(h.NM), nb = (h.NM + bw - 1) / bw, nj = h.NM - (nb - 1) * bw;
  return (size_t)(f64_base(nb - 1, bw) + h.NM * f64_ld(nj)) * 8;
}

// the four-index form pays when it needs fewer products than the Cholesky form
// ((N M)^2 / 2 against X N^2 M per walker and spin, i.e. M < 2 X), the system
// is large enough for its set-up to matter, and its planes take at most a
// quarter of the free device memory (the set-up transients half)
bool eri_pays(afq_system s) {
  if (2L * s->X <= s->M) return false;
  size_t bytes = 0;
  for (int sp = 0; sp < (s->n_up == s->n_dn ? 1 : 2); ++sp) {
    const Shape h = shape_of(s, sp);
    if (h.NM < 4096) return false;
    bytes += tensor_bytes_of(h, s->prec);
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return false;
  const long nm = std::max(shape_of(s, 0).NM, shape_of(s, 1).NM);
  // set-up transients: Lt transposed and one column slab of the Gram matrix
  const size_t transient = (size_t)nm * s->X * 8 + (size_t)s->M * nm * 8;
  return bytes <= free_b / 4 && bytes + transient <= free_b / 2;
}

// W'' planes and work units of both spins (one copy when the two trial blocks are equal)
int eri_prepare(afq_system s) {
  hipStream_t st = s->stream;
  const int M = s->M, X = s->X, ntot = s->ntot;
  AFQ_CHECK(s->LtRe.p, AFQ_E_STATE, "exchange (four-index): real half-rotated vectors missing");
  bool same = s->n_up == s->n_dn;
  if (same) {
    std::vector<double2> ph((size_t)M * ntot);
    AFQ_TRY_HIP(hipMemcpyAsync(ph.data(), s->phi.p, ph.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    AFQ_TRY_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < M && same; ++i)
      for (int a = 0; a < s->n_up && same; ++a) {
        const double2 x = ph[(size_t)i * ntot + a], y = ph[(size_t)i * ntot + s->n_up + a];
        same = x.x == y.x && x.y == y.y;
      }
  }
  s->eri_share = same;
  for (int sp = 0; sp < (same ? 1 : 2); ++sp) {
    const int off = s->spin_off(sp);
    const Shape h = shape_of(s, sp);
    AFQ_CHECK(h.NM <= 65535L * 32, AFQ_E_UNSUPPORTED, "exchange (four-index): N M too large");
    const bool f64 = s->prec == AFQ_FP64;
    const std::vector<int> units = f64 ? std::vector<int>() : make_units(h, choose_interval(h));
    DevBuf LT, SL;
    int rc = s->eri_w[sp].alloc(tensor_bytes_of(h, s->prec));
    if (rc == AFQ_OK) rc = LT.alloc((size_t)h.NM * X * 8);
    if (rc == AFQ_OK) rc = SL.alloc((size_t)M * h.NM * 8);
    if (rc == AFQ_OK && !f64) rc = s->eri_units[sp].alloc(units.size() * sizeof(int));
    if (rc == AFQ_OK) {
      // LT[(a,k)][n] = Lt_n[a][k]
      hipLaunchKernelGGL(transpose_real_kernel, dim3(grid_of((long)X * h.NM)), dim3(256), 0, st,
                         s->LtRe.as<double>() + (long)off * M, (long)X, h.NM, (long)ntot * M, LT.as<double>());
      rc = hip_status(hipGetLastError(), "exchange (four-index): transpose");
    }
    const int N = s->nspin_n(sp);
    const long bw = blk64(h.NM);
    for (int a = 0; a < N && rc == AFQ_OK; ++a) {
      // rows the stored triangle keeps in the slab's columns [a M, a M + M)
      const long j_lo = (long)a * M, j_hi = j_lo + M;
      const long c_first = j_lo / KC, c_last = (j_hi - 1) / KC;
      const long rmax = f64 ? std::min(h.NM, ((j_hi - 1) / bw + 1) * bw) : tri_rows(c_last);
      const long n = (std::min(rmax, h.NM) + M - 1) / M * M;
      // SL[k][(b,l)] = sum_n LT[(a,k)][n] LT[(b,l)][n], b < n / M
      GemmArgs<double> g = gemm_args<double>();
      g.m = M; g.n = (int)n; g.k = X;
      g.A = LT.as<double>() + j_lo * X; g.lda = X; g.cA = false;
      g.B = LT.as<double>(); g.ldb = X; g.opB = OP_T; g.cB = false;
      g.C = SL.as<double>(); g.ldc = n; g.cC = false;
      rc = gemm<double>(g, st);
      if (rc != AFQ_OK) break;
      if (f64) {
        hipLaunchKernelGGL(eri_pack_slab_f64_kernel, dim3(grid_of(rmax * M)), dim3(256), 0, st, SL.as<double>(), n,
                           M, h.NM, a, bw, rmax, s->eri_w[sp].as<double>());
      } else {
        unsigned short* hi = s->eri_w[sp].as<unsigned short>();
        const int ncs = (int)(c_last - c_first + 1);
        hipLaunchKernelGGL(eri_pack_slab_kernel, dim3(grid_of(ncs * rmax * KC)), dim3(256), 0, st, SL.as<double>(),
                           n, M, h.NM, a, c_first, ncs, rmax, (int)(a == N - 1), hi, hi + plane_a_bytes(h) / 2);
      }
      rc = hip_status(hipGetLastError(), "exchange (four-index): pack");
    }
    if (rc == AFQ_OK && !f64)
      rc = hip_status(hipMemcpyAsync(s->eri_units[sp].p, units.data(), units.size() * sizeof(int),
                                     hipMemcpyHostToDevice, st),
                      "exchange (four-index): units");
    // SL and LT are freed on return: wait for the kernels that read them
    if (rc == AFQ_OK) rc = hip_status(hipStreamSynchronize(st), "exchange (four-index): set-up");
    if (rc != AFQ_OK) {
      (void)hipStreamSynchronize(st);
      eri_free(s);
      return rc;
    }
    s->eri_nunit[sp] = (int)(units.size() / 4);
    s->eri_units_host[sp] = units;
  }
  ++s->eri_gen;
  s->eri_ready = true;
  s->eri_prec = s->prec;
  return AFQ_OK;
}

}  // namespace

int eri_sync(afq_system s) {
  const bool can = s->kp_nk == 0 && s->msd_n == 0 && (s->prec == AFQ_BF16X3 || s->prec == AFQ_FP64) &&
                   s->real_trial && s->eri_form != AFQ_EXCH_CHOLESKY;
  if (!can || (s->eri_ready && s->eri_prec != s->prec)) {
    if (s->eri_ready) {
      eri_free(s);
      ++s->version;
    }
    if (!can) return AFQ_OK;
  }
  if (s->eri_ready) return AFQ_OK;
  if (s->eri_form == AFQ_EXCH_AUTO) {
    if (s->eri_declined) return AFQ_OK;
    if (!eri_pays(s)) {
      s->eri_declined = true;
      return AFQ_OK;
    }
  }
  AFQ_RET(eri_prepare(s));
  ++s->version;
  return AFQ_OK;
}

size_t eri_tensor_bytes(afq_system s) { return s->eri_w[0].bytes + s->eri_w[1].bytes; }

// spins contracted per launch: both when they share the tensor (one pass over
// W'' for twice the columns), else one
static int eri_nsp(afq_system s) { return s->eri_share ? 2 : 1; }

int eri_alloc_scratch(afq_system s, afq_walkers w) {
  if (!s->eri_ready) return AFQ_OK;
  if (s->eri_prec == AFQ_FP64) {   // Z^T of one spin at a time
    const size_t zb = (size_t)w->nw * std::max(shape_of(s, 0).NM, shape_of(s, 1).NM) * sizeof(double2);
    if (w->eri_part.bytes < zb) AFQ_RET(w->eri_part.alloc(zb));
    return AFQ_OK;
  }
  const long rows_b = rows_b_of(eri_nsp(s) * w->nw);
  size_t tb = 0, pb = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const Shape h = shape_of(s, sp);
    tb = std::max(tb, 2 * plane_bytes(rows_b, h.nchunk));
    pb = std::max(pb, (size_t)s->eri_nunit[s->eri_share ? 0 : sp] * rows_b * sizeof(double2));
  }
  if (w->eri_theta.bytes < tb) AFQ_RET(w->eri_theta.alloc(tb));
  if (w->eri_part.bytes < pb) AFQ_RET(w->eri_part.alloc(pb));
  // launch layouts of the tensor blocks (rebuilt when the units or the
  // column blocks change; outside any step, so the upload may synchronise)
  const int nblk_b = (int)(rows_b / RBR);
  const long key = (long)s->eri_gen * 65536 + nblk_b;
  bool uploaded = false;
  for (int wsp = 0; wsp < (s->eri_share ? 1 : 2); ++wsp) {
    if (w->eri_wg_key[wsp] == key) continue;
    std::vector<int>& lay = w->eri_wg_host[wsp];
    lay = make_wg_layout(s->eri_units_host[wsp], shape_of(s, wsp).nblk_a, nblk_b);
    {   // every (unit, column block) exactly once
      const long nu = (long)s->eri_units_host[wsp].size() / 4;
      std::vector<char> seen((size_t)(nu * nblk_b), 0);
      long n = 0;
      for (size_t i = 0; i + 1 < lay.size(); i += 2) {
        if (lay[i] < 0) continue;
        const long k = (long)lay[i] * nblk_b + lay[i + 1];
        AFQ_CHECK(lay[i] < nu && lay[i + 1] >= 0 && lay[i + 1] < nblk_b && !seen[k], AFQ_E_STATE,
                  "exchange (four-index): launch layout");
        seen[k] = 1;
        ++n;
      }
      AFQ_CHECK(n == nu * nblk_b, AFQ_E_STATE, "exchange (four-index): launch layout incomplete");
    }
    AFQ_RET(w->eri_wg[wsp].alloc(lay.size() * sizeof(int)));
    AFQ_TRY_HIP(hipMemcpyAsync(w->eri_wg[wsp].p, lay.data(), lay.size() * sizeof(int), hipMemcpyHostToDevice,
                               s->stream));
    w->eri_wg_launch[wsp] = (int)(lay.size() / 2);
    w->eri_wg_key[wsp] = key;
    uploaded = true;
  }
  if (uploaded) AFQ_TRY_HIP(hipStreamSynchronize(s->stream));
  return AFQ_OK;
}

int eri_pack(afq_system s, afq_walkers w, int sp, hipStream_t st) {
  if (s->eri_prec == AFQ_FP64) return AFQ_OK;   // the GEMMs read Theta^T in place
  const Shape h = shape_of(s, sp);
  const int nsp = eri_nsp(s);
  const long rows_b = rows_b_of(nsp * w->nw);
  const size_t pb = plane_bytes(rows_b, h.nchunk);
  AFQ_CHECK(s->eri_ready && w->eri_theta.bytes >= 2 * pb, AFQ_E_STATE,
            "exchange (four-index): walker scratch not prepared");
  AFQ_CHECK(nsp == 1 || sp == 0, AFQ_E_INVALID, "exchange (four-index): shared tensor packs both spins at once");
  unsigned short* th = w->eri_theta.as<unsigned short>();
  hipLaunchKernelGGL(eri_pack_theta_kernel, dim3(grid_of((long)h.nchunk * (rows_b / 2) * KC)), dim3(256), 0, st,
                     w->theta.as<double2>(), s->ntot, s->M, s->spin_off(sp), s->spin_off(1), nsp, (int)h.NM, w->nw,
                     rows_b, h.nchunk, th, th + pb / 2);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// out[w * ld_out] = sum_{i < n} a[w * lda + i] z[w * ldz + i] (complex, no
// conjugate), one 256-thread workgroup per walker, fixed-order tree; the
// entries 1..X-1 after it are zeroed (the assembly sums over all X entries)
__global__ __launch_bounds__(256) void cdot_rows_kernel(const double2* __restrict__ a, long lda,
                                                        const double2* __restrict__ z, long ldz, long n,
                                                        double2* __restrict__ out, long ld_out, int X) {
  __shared__ double2 red[256];
  const int w = blockIdx.x, t = threadIdx.x;
  const double2* aw = a + (long)w * lda;
  const double2* zw = z + (long)w * ldz;
  double2 acc = make_double2(0.0, 0.0);
  for (long i = t; i < n; i += 256) acc = cadd(acc, cmul(aw[i], zw[i]));
  red[t] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] = cadd(red[t], red[t + h]);
    __syncthreads();
  }
  double2* o = out + (long)w * ld_out;
  if (t == 0) o[0] = red[0];
  for (int k = 1 + t; k < X; k += 256) o[k] = make_double2(0.0, 0.0);
}

static int launch_cdot_rows(const double2* a, long lda, const double2* z, long ldz, long n, int nw, double2* out,
                            long ld_out, int X, hipStream_t st) {
  hipLaunchKernelGGL(cdot_rows_kernel, dim3(nw), dim3(256), 0, st, a, lda, z, ldz, n, out, ld_out, X);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// FP64 form, one spin: Z^T (nw x NM) over the column blocks, then the dot products
static int eri_exchange_f64(afq_system s, afq_walkers w, int sp, hipStream_t st) {
  const Shape h = shape_of(s, sp);
  const int wsp = s->eri_share ? 0 : sp;
  const long NM = h.NM, ldt = (long)s->ntot * s->M;
  AFQ_CHECK(s->eri_ready && s->eri_w[wsp].bytes >= tensor_bytes_of(h, AFQ_FP64), AFQ_E_STATE,
            "exchange (four-index, FP64): tensor not prepared");
  AFQ_CHECK(w->eri_part.bytes >= (size_t)w->nw * NM * sizeof(double2), AFQ_E_STATE,
            "exchange (four-index, FP64): walker scratch not prepared");
  const double* Wt = s->eri_w[wsp].as<double>();
  const double* th = w->theta.as<double>() + 2L * s->spin_off(sp) * s->M;   // row w: Theta-hat of walker w
  double* Z = w->eri_part.as<double>();
  const long bw = blk64(NM);
  for (long j0 = 0, jb = 0; j0 < NM; j0 += bw, ++jb) {
    const long nj = std::min(bw, NM - j0);
    const double* col = Wt + f64_base(jb, bw);   // block column J: rows 0 .. j0 + nj, ld f64_ld(nj)
    GemmArgs<double> g = gemm_args<double>();
    g.m = w->nw; g.n = (int)nj;
    g.A = th; g.lda = ldt; g.cA = true;
    g.ldb = f64_ld(nj); g.cB = false;
    g.C = Z + 2 * j0; g.ldc = NM; g.cC = true;
    // Z_J = Theta-hat_J^T W'_JJ
    g.k = (int)nj;
    g.A = th + 2 * j0;
    g.B = col + j0 * g.ldb;
    AFQ_RET(gemm<double>(g, st));
    if (j0 > 0) {   // Z_J += 2 Theta-hat_{<J}^T W'_{<J,J}
      g.k = (int)j0;
      g.A = th;
      g.B = col;
      g.ar = 2.0; g.ai = 0.0; g.br = 1.0; g.bi = 0.0;
      AFQ_RET(gemm<double>(g, st));
    }
  }
  return launch_cdot_rows(reinterpret_cast<const double2*>(th), ldt, reinterpret_cast<const double2*>(Z), NM,
                          NM, w->nw, w->troo.as<double2>() + (long)sp * s->X, 2L * s->X, s->X, st);
}

int eri_exchange(afq_system s, afq_walkers w, int sp, hipStream_t st) {
  if (s->eri_prec == AFQ_FP64) {
    for (int q = 0; q < eri_nsp(s); ++q) AFQ_RET(eri_exchange_f64(s, w, sp + q, st));
    return AFQ_OK;
  }
  const Shape h = shape_of(s, sp);
  const int wsp = s->eri_share ? 0 : sp;
  const int nsp = eri_nsp(s);
  AFQ_CHECK(nsp == 1 || sp == 0, AFQ_E_INVALID, "exchange (four-index): shared tensor contracts both spins at once");
  const long rows_b = rows_b_of(nsp * w->nw);
  const size_t pa = plane_a_bytes(h), pb = plane_bytes(rows_b, h.nchunk);
  const int nunit = s->eri_nunit[wsp];
  AFQ_CHECK(s->eri_ready && nunit > 0 && s->eri_w[wsp].bytes >= 2 * pa, AFQ_E_STATE,
            "exchange (four-index): tensor not prepared");
  AFQ_CHECK(w->eri_theta.bytes >= 2 * pb && w->eri_part.bytes >= (size_t)nunit * rows_b * sizeof(double2),
            AFQ_E_STATE, "exchange (four-index): walker scratch not prepared");
  EriArgs g{};
  g.a[0] = s->eri_w[wsp].as<unsigned char>();
  g.a[1] = g.a[0] + pa;
  g.b[0] = w->eri_theta.as<unsigned char>();
  g.b[1] = g.b[0] + pb;
  g.rows_b = rows_b;
  g.units = s->eri_units[wsp].as<int4>();
  AFQ_CHECK(w->eri_wg_key[wsp] == (long)s->eri_gen * 65536 + rows_b / RBR && w->eri_wg_launch[wsp] > 0,
            AFQ_E_STATE, "exchange (four-index): launch layout not prepared");
  g.wg = w->eri_wg[wsp].as<int2>();
  g.thetaT = w->theta.as<double2>();
  g.ntot = s->ntot; g.M = s->M; g.off = s->spin_off(sp); g.NM = (int)h.NM; g.nw = w->nw;
  g.off1 = s->spin_off(1); g.nsp = nsp;
  g.part = w->eri_part.as<double2>();
  hipLaunchKernelGGL(eri_kernel, dim3((unsigned)w->eri_wg_launch[wsp]), dim3(256), 0, st, g);
  AFQ_TRY_HIP(hipGetLastError());
  for (int q = 0; q < nsp; ++q) {   // spin sp + q: columns 2 (q nw + w) + part
    hipLaunchKernelGGL(eri_reduce_kernel, dim3(w->nw), dim3(256), 0, st, w->eri_part.as<double2>() + 2L * q * w->nw,
                       nunit, rows_b, w->nw, sp + q, s->X, w->troo.as<double2>());
    AFQ_TRY_HIP(hipGetLastError());
  }
  return AFQ_OK;
}
