// FP32 contractions of the reduced-precision modes on v_mfma_f32_16x16x4f32,
// streamed through the three-stage direct global->LDS ring:
//
//   * the propagator matrices A_w = sum_n c_wn L^n: coefficient rows
//     (w, Re|Im) times the Cholesky vectors, which are packed once per system
//     k-contiguous (entry e of L^n at [n / 16][e][n % 16]); the epilogue writes
//     A_w as complex FP32;
//   * the force-bias traces tr(Lt^{ns} Theta^s) = sum_(a,k) Theta-hat[(a,k)] Lt_n[a][k]
//     (split-BF16x3 mode, real trial): Theta-hat rows (w, Re|Im) times the
//     real half-rotated vectors, packed once per system; the N M contraction is
//     split into runs whose FP32 tiles are summed in FP64 in a fixed order.
//
// Both are C = A B^T with A and B packed chunk-major (64-byte rows of 16 FP32
// contraction elements, all rows of a chunk contiguous), the same layout and
// swizzle as the split-BF16x3 kernels. Workgroup tile 256 x 128 (2 x 2 waves
// of 8 x 4 MFMA tiles), 72 KB of LDS, two workgroups per CU.
#include <algorithm>
#include "common.h"
#include "mfma_ring.h"

namespace {

using ring::f4;
using ring::lds_t;
using ring::ROWB;
using ring::swz;
using ring::wait_vm_barrier;

constexpr int NWAVE = 4, NXCD = 8;
constexpr int RK = 16;                      // FP32 contraction elements per chunk row
constexpr int TA = 8, TB = 4;
constexpr int RA = 32 * TA, RBR = 32 * TB;  // 256 x 128
constexpr int REGA = RA * ROWB, REGB = RBR * ROWB;
constexpr int STAGE = REGA + REGB;
constexpr int NT = STAGE / 1024, NQ = NT / NWAVE;
static_assert(NT % NWAVE == 0, "loads must split evenly over the waves");

enum { EPI_AMAT = 0, EPI_PART = 1 };

struct R32Args {
  const unsigned char* a;   // packed A: [chunk][rows_a][16] float
  const unsigned char* b;   // packed B: [chunk][rows_b][16] float
  long rows_a, rows_b;
  int nchunk, kper, nblk_a, nblk_b;
  int nunit, grid;          // units = A row blocks x contraction runs; grid = units x B blocks
  int a_fast;               // 1: consecutive workgroups take consecutive A row blocks (sharing a B block)
  float2* amat;             // EPI_AMAT: rows (w, Re|Im), columns e -> amat[w][e]
  long ncol;
  int nw;
  float* part;              // EPI_PART: part[(run * rows_a + row) * rows_b + col]
};

template <int EPI>
__global__ __launch_bounds__(256, 2) void ring32_kernel(R32Args g) {
  __shared__ __align__(16) unsigned char L0[STAGE];
  __shared__ __align__(16) unsigned char L1[STAGE];
  __shared__ __align__(16) unsigned char L2[STAGE];
  __shared__ float trash[NWAVE * 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rb = wave >> 1, cb = wave & 1;
  // XCD-aware order: workgroup i runs on XCD i % 8; each XCD takes a
  // contiguous range of the logical order
  const int per = (int)(gridDim.x / NXCD);
  const int lid = (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
  if (lid >= g.grid) return;
  int u, bb;
  if (g.a_fast) {
    u = lid % g.nunit;
    bb = lid / g.nunit;
  } else {
    u = lid / g.nblk_b;
    bb = lid - u * g.nblk_b;
  }
  const int p = u % g.nblk_a, run = u / g.nblk_a;
  const int c0 = run * g.kper, nc = min(g.kper, g.nchunk - c0);   // >= 1
  const long arow0 = (long)p * RA, brow0 = (long)bb * RBR;
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
    src[q] = (isb ? g.b : g.a) + ((isb ? brow0 : arow0) + row) * ROWB + 16 * c + (long)c0 * cstride[q];
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
  const int arow = rb * (RA / 2), brow = cb * (RBR / 2);
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
  if constexpr (EPI == EPI_AMAT) {
#pragma unroll
    for (int i = 0; i < TA; ++i)
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        const long row0 = arow0 + arow + 16 * i + 4 * lq;    // rows (w0, Re), (w0, Im), (w0 + 1, Re), (w0 + 1, Im)
        const long col = brow0 + brow + 16 * j + lr;
        const int w0 = (int)(row0 >> 1);
        if (col < g.ncol) {
          if (w0 < g.nw) g.amat[(long)w0 * g.ncol + col] = make_float2(acc[i][j][0], acc[i][j][1]);
          if (w0 + 1 < g.nw) g.amat[(long)(w0 + 1) * g.ncol + col] = make_float2(acc[i][j][2], acc[i][j][3]);
        }
      }
  } else {
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

// columns of a row-major matrix as rows of a packed operand (the Cholesky
// vectors, k = vector index): out[(c rows + e) 16 + kk] = src[(16 c + kk) ncol + e]
__global__ void pack_cols_kernel(const double* __restrict__ src, long ncol, int K, long rows, int nchunk,
                                 float* __restrict__ out) {
  const long total = (long)nchunk * rows * RK;
  for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    // consecutive threads read consecutive e of one vector
    const long k = t / rows, e = t - k * rows;
    const float v = (k < K && e < ncol) ? (float)src[k * ncol + e] : 0.f;
    out[((k / RK) * rows + e) * RK + (k % RK)] = v;
  }
}

// tro[w][spin][n] = sum over runs (fixed order) of (part[run][2w][n], part[run][2w + 1][n])
__global__ void coulomb_reduce_kernel(const float* __restrict__ part, int nrun, long rows_a, long rows_b, int nw,
                                      int X, int spin, double2* __restrict__ tro) {
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
}

int grid_of(long total) { return (int)std::min<long>(std::max<long>((total + 255) / 256, 1), 1 << 20); }
long pad_to(long x, long m) { return (x + m - 1) / m * m; }

template <int EPI>
int launch(R32Args& g, hipStream_t st) {
  g.nblk_a = (int)(g.rows_a / RA);
  g.nblk_b = (int)(g.rows_b / RBR);
  const int nrun = (g.nchunk + g.kper - 1) / g.kper;
  const long nunit = (long)g.nblk_a * nrun, grid = nunit * g.nblk_b;
  AFQ_CHECK(g.nchunk >= 1 && g.rows_a % RA == 0 && g.rows_b % RBR == 0 && grid < (1L << 30), AFQ_E_INVALID,
            "FP32 ring contraction: bad shape");
  g.nunit = (int)nunit;
  g.grid = (int)grid;
  const long launch = (grid + NXCD - 1) / NXCD * NXCD;
  hipLaunchKernelGGL(ring32_kernel<EPI>, dim3((unsigned)launch), dim3(256), 0, st, g);
  return hip_status(hipGetLastError(), "FP32 ring contraction");
}

// rows of the coefficient operand and of the Theta-hat operand for nw walkers
long coef_rows(int nw) { return pad_to(2L * nw, RA); }

// runs of the force-bias contraction: about 2048 workgroups, runs of at least 16 chunks
int coulomb_kper(long nchunk, long rows_a, long rows_b) {
  const long tiles = (rows_a / RA) * (rows_b / RBR);
  const long nrun = std::max<long>(1, std::min<long>(nchunk / 16, (2048 + tiles - 1) / tiles));
  return (int)((nchunk + nrun - 1) / nrun);
}

}  // namespace

bool r32_coulomb_used(afq_system s) { return s->lt32[0].p != nullptr; }

int r32_prepare(afq_system s) {
  hipStream_t st = s->stream;
  const bool reduced = s->prec != AFQ_FP64 && s->kp_nk == 0;
  if (reduced && !s->chol32t.p) {
    const long m2 = (long)s->M * s->M;
    const long rows = pad_to(m2, RBR);
    const int nchunk = (int)pad_to(s->X, RK) / RK;
    AFQ_RET(s->chol32t.alloc((size_t)nchunk * rows * RK * sizeof(float)));
    hipLaunchKernelGGL(pack_cols_kernel, dim3(grid_of((long)nchunk * rows * RK)), dim3(256), 0, st,
                       s->chol.as<double>(), m2, s->X, rows, nchunk, s->chol32t.as<float>());
    AFQ_TRY_HIP(hipGetLastError());
  }
  const bool coul = s->prec == AFQ_BF16X3 && s->real_trial && s->kp_nk == 0 && s->msd_n == 0;
  if (coul && !s->lt32[0].p) {
    AFQ_CHECK(s->LtRe.p, AFQ_E_STATE, "force bias (FP32 ring): real half-rotated vectors missing");
    for (int sp = 0; sp < 2; ++sp) {
      const long NM = (long)s->nspin_n(sp) * s->M;
      const long rows = pad_to(s->X, RBR);
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
  }
  if (!reduced && s->chol32t.p) s->chol32t.free();
  return AFQ_OK;
}

int r32_alloc_scratch(afq_system s, afq_walkers w) {
  if (!s->chol32t.p) return AFQ_OK;
  const long rows = coef_rows(w->nw);
  size_t cb = (size_t)(pad_to(s->X, RK)) * rows * sizeof(float);
  if (w->r32_coef.bytes < cb) AFQ_RET(w->r32_coef.alloc(cb));
  if (!s->lt32[0].p) return AFQ_OK;
  size_t tb = 0, pb = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const long NM = (long)s->nspin_n(sp) * s->M;
    const long nchunk = pad_to(NM, RK) / RK, rows_b = pad_to(s->X, RBR);
    tb = std::max(tb, (size_t)nchunk * rows * RK * sizeof(float));
    const int kper = coulomb_kper(nchunk, rows, rows_b);
    const long nrun = (nchunk + kper - 1) / kper;
    pb = std::max(pb, (size_t)nrun * rows * rows_b * sizeof(float));
  }
  if (w->r32_theta.bytes < tb) AFQ_RET(w->r32_theta.alloc(tb));
  if (w->r32_part.bytes < pb) AFQ_RET(w->r32_part.alloc(pb));
  return AFQ_OK;
}

int r32_abuild(afq_system s, afq_walkers w, const float* coef, float2* amat, hipStream_t st) {
  const long rows = coef_rows(w->nw);
  const int nchunk = (int)(pad_to(s->X, RK) / RK);
  AFQ_CHECK(s->chol32t.p && w->r32_coef.bytes >= (size_t)nchunk * rows * RK * sizeof(float), AFQ_E_STATE,
            "propagator build (FP32 ring): operands not prepared");
  hipLaunchKernelGGL(pack_cplx_rows_kernel<float>, dim3(grid_of((long)nchunk * rows * RK)), dim3(256), 0, st, coef,
                     (long)s->X, w->nw, (long)s->X, rows, nchunk, w->r32_coef.as<float>());
  AFQ_TRY_HIP(hipGetLastError());
  R32Args g{};
  g.a = w->r32_coef.as<unsigned char>();
  g.b = s->chol32t.as<unsigned char>();
  g.rows_a = rows;
  g.rows_b = pad_to((long)s->M * s->M, RBR);
  g.nchunk = nchunk;
  g.kper = nchunk;
  g.a_fast = 1;
  g.amat = amat;
  g.ncol = (long)s->M * s->M;
  g.nw = w->nw;
  return launch<EPI_AMAT>(g, st);
}

int r32_coulomb(afq_system s, afq_walkers w, hipStream_t st) {
  AFQ_CHECK(s->lt32[0].p, AFQ_E_STATE, "force bias (FP32 ring): operands not prepared");
  const long rows = coef_rows(w->nw), rows_b = pad_to(s->X, RBR);
  for (int sp = 0; sp < 2; ++sp) {
    const long NM = (long)s->nspin_n(sp) * s->M;
    const int nchunk = (int)(pad_to(NM, RK) / RK);
    const int kper = coulomb_kper(nchunk, rows, rows_b);
    const int nrun = (nchunk + kper - 1) / kper;
    AFQ_CHECK(w->r32_theta.bytes >= (size_t)nchunk * rows * RK * sizeof(float) &&
                  w->r32_part.bytes >= (size_t)nrun * rows * rows_b * sizeof(float),
              AFQ_E_STATE, "force bias (FP32 ring): walker scratch not prepared");
    // Theta-hat rows (w, Re|Im): thetaT[w][off + a][k] at (a, k) -> a M + k
    hipLaunchKernelGGL(pack_cplx_rows_kernel<double>, dim3(grid_of((long)nchunk * rows * RK)), dim3(256), 0, st,
                       reinterpret_cast<const double*>(w->theta.as<double2>() + (long)s->spin_off(sp) * s->M),
                       (long)s->ntot * s->M, w->nw, NM, rows, nchunk, w->r32_theta.as<float>());
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
    AFQ_RET(launch<EPI_PART>(g, st));
    hipLaunchKernelGGL(coulomb_reduce_kernel, dim3(grid_of((long)w->nw * s->X)), dim3(256), 0, st,
                       w->r32_part.as<float>(), nrun, rows, rows_b, w->nw, s->X, sp, w->tro.as<double2>());
    AFQ_TRY_HIP(hipGetLastError());
  }
  return AFQ_OK;
}
