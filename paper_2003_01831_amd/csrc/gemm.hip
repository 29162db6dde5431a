// Batched complex/real GEMM on MFMA for the medium contractions of the walker
// step (B1 W, the Taylor products A V, the A = sum_n c_n L^n build, the FP64
// force-bias traces, the multi-determinant and adjoint products and the system
// set-up; the overlaps, Theta and the CholeskyQR products have their own
// kernels in overlap.hip):
//
//   C = alpha op(A) op(B) + beta C,   optionally D += alpha op(A) op(B)
//
// 64 x 64 output tile per 256-thread workgroup; each wave owns a 32 x 32
// quarter as 2 x 2 MFMA tiles (v_mfma_f64_16x16x4f64 or
// v_mfma_f32_16x16x4f32). A complex product is four real MFMAs
// (Re += ar br - ai bi, Im += ar bi + ai br); a real operand drops the terms
// of its imaginary part at compile time. k is staged through LDS in chunks of
// 16 as separate Re/Im planes, k-major so that fragment reads are contiguous.
// Long contractions with few output tiles are split over k into a workspace
// and reduced in a fixed order (deterministic).
#include <map>
#include <mutex>
#include "common.h"

namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 4;

typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(4))) double d4;

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using Acc = d4;
  __device__ static void mma(Acc& c, double a, double b) { c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  using Acc = f4;
  __device__ static void mma(Acc& c, float a, float b) { c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

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

// ksplit > 1: blockIdx.z = batch * ksplit + split; the partial products of a
// split go to ws[(batch * ksplit + split)][m][n] (complex T) instead of C/D.
template <typename T, bool CA, bool CB>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(GemmArgs<T> g, int ksplit, int kchunk, T* ws) {
  using M = Mfma<T>;
  using Acc = typename M::Acc;
  constexpr bool CPLX = CA || CB;
  __shared__ T As_r[BK][BM + PAD], Bs_r[BK][BN + PAD];
  __shared__ T As_i[CA ? BK : 1][BM + PAD], Bs_i[CB ? BK : 1][BN + PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long b = blockIdx.z / ksplit;
  const int split = blockIdx.z - (int)b * ksplit;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const T* A = g.A + b * g.sA * (CA ? 2 : 1);
  const T* B = g.B + b * g.sB * (CB ? 2 : 1);
  const bool ca = g.opA == OP_C || g.opA == OP_R, cb = g.opB == OP_C || g.opB == OP_R;
  const bool na = g.opA == OP_N || g.opA == OP_R, nb = g.opB == OP_N || g.opB == OP_R;   // untransposed
  const int kbeg = split * kchunk, kend = min(g.k, kbeg + kchunk);

  Acc acc_r[2][2], acc_i[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) { acc_r[i][j][r] = 0; acc_i[i][j][r] = 0; }

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int e = tid + 256 * rr;
      int kk, mm;
      if (na) { kk = e & 15; mm = e >> 4; } else { kk = e >> 6; mm = e & 63; }
      const int gi = m0 + mm, gk = k0 + kk;
      T re = T(0), im = T(0);
      if (gi < g.m && gk < kend) {
        const long idx = na ? (long)gi * g.lda + gk : (long)gk * g.lda + gi;
        load_elem(A, idx, CA, ca, re, im);
      }
      As_r[kk][mm] = re;
      if constexpr (CA) As_i[kk][mm] = im;
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int e = tid + 256 * rr;
      int kk, nn;
      if (nb) { kk = e >> 6; nn = e & 63; } else { kk = e & 15; nn = e >> 4; }
      const int gj = n0 + nn, gk = k0 + kk;
      T re = T(0), im = T(0);
      if (gj < g.n && gk < kend) {
        const long idx = nb ? (long)gk * g.ldb + gj : (long)gj * g.ldb + gk;
        load_elem(B, idx, CB, cb, re, im);
      }
      Bs_r[kk][nn] = re;
      if constexpr (CB) Bs_i[kk][nn] = im;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4), c16 = lane & 15;
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ar[t] = As_r[kr][wm * 32 + t * 16 + c16];
        br[t] = Bs_r[kr][wn * 32 + t * 16 + c16];
        if constexpr (CA) ai[t] = As_i[kr][wm * 32 + t * 16 + c16];
        if constexpr (CB) bi[t] = Bs_i[kr][wn * 32 + t * 16 + c16];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          M::mma(acc_r[i][j], ar[i], br[j]);
          if constexpr (CA && CB) M::mma(acc_r[i][j], -ai[i], bi[j]);
          if constexpr (CB) M::mma(acc_i[i][j], ar[i], bi[j]);
          if constexpr (CA) M::mma(acc_i[i][j], ai[i], br[j]);
        }
    }
    __syncthreads();
  }

  if (ksplit > 1) {
    T* w = ws + ((long)blockIdx.z * g.m * g.n) * 2;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = m0 + wm * 32 + i * 16 + M::row(lane, r);
          const int gj = n0 + wn * 32 + j * 16 + (lane & 15);
          if (gi < g.m && gj < g.n) {
            w[2 * ((long)gi * g.n + gj)] = acc_r[i][j][r];
            w[2 * ((long)gi * g.n + gj) + 1] = CPLX ? acc_i[i][j][r] : T(0);
          }
        }
    return;
  }
  T* C = g.C ? g.C + b * g.sC * (g.cC ? 2 : 1) : nullptr;
  double2* D = g.D ? g.D + b * g.sD : nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm * 32 + i * 16 + M::row(lane, r);
        const int gj = n0 + wn * 32 + j * 16 + (lane & 15);
        if (gi >= g.m || gj >= g.n) continue;
        const double xr = (double)acc_r[i][j][r], xi = CPLX ? (double)acc_i[i][j][r] : 0.0;
        double vr = g.ar * xr - g.ai * xi;
        double vi = g.ar * xi + g.ai * xr;
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

// fixed-order sum of the k splits, then the same epilogue as the kernel above
template <typename T>
__global__ void gemm_splitk_reduce(GemmArgs<T> g, int ksplit, const T* ws) {
  const long mn = (long)g.m * g.n;
  const long total = mn * g.batch;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long b = t / mn, e = t - b * mn;
    const int gi = (int)(e / g.n), gj = (int)(e - (long)gi * g.n);
    double xr = 0.0, xi = 0.0;
    for (int s = 0; s < ksplit; ++s) {
      const T* w = ws + ((b * ksplit + s) * mn + e) * 2;
      xr += (double)w[0];
      xi += (double)w[1];
    }
    double vr = g.ar * xr - g.ai * xi;
    double vi = g.ar * xi + g.ai * xr;
    if (g.C) {
      T* C = g.C + b * g.sC * (g.cC ? 2 : 1);
      const long ci = (long)gi * g.ldc + gj;
      if (g.br != 0.0 || g.bi != 0.0) {
        double cr, cim;
        if (g.cC) { cr = C[2 * ci]; cim = C[2 * ci + 1]; } else { cr = C[ci]; cim = 0.0; }
        vr += g.br * cr - g.bi * cim;
        vi += g.br * cim + g.bi * cr;
      }
      if (g.cC) { C[2 * ci] = (T)vr; C[2 * ci + 1] = (T)vi; } else { C[ci] = (T)vr; }
    }
    if (g.D) {
      double2* d = g.D + b * g.sD + (long)gi * g.ldd + gj;
      d->x += vr;
      d->y += vi;
    }
  }
}

// ---------------------------------------------------------------------------
// Tiled path for the large contractions (A row-major with k contiguous, B
// either n-contiguous or k-contiguous): a (32 WM) x (32 WN) tile per 256-thread
// workgroup, each wave a WM x WN grid of 16 x 16 MFMA tiles. k advances in
// chunks of 16: the next chunk is fetched from HBM into registers with 16-byte
// loads while the current one is multiplied out of LDS. LDS planes hold Re and
// Im separately; rows of k-contiguous planes are padded so that both the
// fragment reads and the 8-byte stores are bank-conflict free. A complex
// product is issued as four sweeps over the tile grid (Re += ar br, Re -= ai bi,
// Im += ar bi, Im += ai br), so consecutive MFMAs never depend on each other.
template <typename T> struct Vec16;
template <> struct Vec16<float> { using V = float4; static constexpr int E = 4; };
template <> struct Vec16<double> { using V = double2; static constexpr int E = 2; };

template <typename T> __device__ inline typename Vec16<T>::V vmake(const T* t);
template <> __device__ inline float4 vmake<float>(const float* t) { return make_float4(t[0], t[1], t[2], t[3]); }
template <> __device__ inline double2 vmake<double>(const double* t) { return make_double2(t[0], t[1]); }

template <typename T> __device__ inline T vget(const typename Vec16<T>::V& v, int e);
template <> __device__ inline float vget<float>(const float4& v, int e) {
  return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}
template <> __device__ inline double vget<double>(const double2& v, int e) { return e == 0 ? v.x : v.y; }

template <typename T, bool CA, bool CB, bool BT, int WM, int WN>
__global__ __launch_bounds__(256) void gemm_tile_kernel(GemmArgs<T> g, int ksplit, int kchunk, T* ws) {
  using M = Mfma<T>;
  using Acc = typename M::Acc;
  using V = typename Vec16<T>::V;
  constexpr int E = Vec16<T>::E;
  constexpr int BMt = 32 * WM, BNt = 32 * WN, BKt = 16;
  constexpr bool CPLX = CA || CB;
  constexpr int SK = BKt + (sizeof(T) == 4 ? 2 : 1);     // row stride of [row][k] planes
  constexpr int SN = BNt + (sizeof(T) == 4 ? 16 : 8);    // row stride of [k][n] planes
  constexpr int PA = CA ? 2 : 1, PB = CB ? 2 : 1;       // planes
  constexpr int VA = BKt * PA / E;                      // 16-byte vectors per A row chunk
  constexpr int TLA = BMt * VA, NLA = (TLA + 255) / 256;   // vectors per chunk, per thread
  constexpr int VBr = BT ? BKt * PB / E : BNt * PB / E; // vectors per B row (n row if BT, k row else)
  constexpr int TLB = (BT ? BNt : BKt) * VBr, NLB = (TLB + 255) / 256;
  __shared__ T As[PA][BMt * SK];
  __shared__ T Bs[PB][BT ? BNt * SK : BKt * SN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long b = blockIdx.z / ksplit;
  const int split = blockIdx.z - (int)b * ksplit;
  const int m0 = blockIdx.y * BMt, n0 = blockIdx.x * BNt;
  const T* A = g.A + b * g.sA * PA;
  const T* B = g.B + b * g.sB * PB;
  const int kbeg = split * kchunk, kend = min(g.k, kbeg + kchunk);

  V ra[NLA], rb[NLB];
  // fetch one k-chunk into registers (zero outside the matrices)
  auto fetch = [&](int kb) {
#pragma unroll
    for (int u = 0; u < NLA; ++u) {
      const int flat = tid + 256 * u, row = flat / VA, v = flat - row * VA;
      if (TLA % 256 && flat >= TLA) break;
      const int gi = m0 + row, gk = kb + v * E / PA;      // first k of the vector
      const long base = ((long)gi * g.lda + gk) * PA;
      if (gi < g.m && gk + E / PA <= kend) {
        ra[u] = *reinterpret_cast<const V*>(A + base);
      } else {
        T t[E];
#pragma unroll
        for (int e = 0; e < E; ++e) t[e] = (gi < g.m && gk + e / PA < kend) ? A[base + e] : T(0);
        ra[u] = vmake<T>(t);
      }
    }
#pragma unroll
    for (int u = 0; u < NLB; ++u) {
      const int flat = tid + 256 * u, r = flat / VBr, v = flat - r * VBr;
      if (TLB % 256 && flat >= TLB) break;
      if constexpr (BT) {   // B stored n-major: row r = n, vector along k
        const int gj = n0 + r, gk = kb + v * E / PB;
        const long base = ((long)gj * g.ldb + gk) * PB;
        if (gj < g.n && gk + E / PB <= kend) {
          rb[u] = *reinterpret_cast<const V*>(B + base);
        } else {
          T t[E];
#pragma unroll
          for (int e = 0; e < E; ++e) t[e] = (gj < g.n && gk + e / PB < kend) ? B[base + e] : T(0);
          rb[u] = vmake<T>(t);
        }
      } else {              // B stored k-major: row r = k, vector along n
        const int gk = kb + r, gj = n0 + v * E / PB;
        const T* Bm = B;
        int jj = gj;
        if (g.vn) {           // virtual columns: member gj / vn (a vector never straddles two)
          const int mb = gj / g.vn;
          jj = gj - mb * g.vn;
          Bm = g.B + (long)mb * g.sB * PB;
        }
        const long base = ((long)gk * g.ldb + jj) * PB;
        if (gk < kend && gj + E / PB <= g.n) {
          rb[u] = *reinterpret_cast<const V*>(Bm + base);
        } else {
          T t[E];
#pragma unroll
          for (int e = 0; e < E; ++e) t[e] = (gk < kend && gj + e / PB < g.n) ? Bm[base + e] : T(0);
          rb[u] = vmake<T>(t);
        }
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int u = 0; u < NLA; ++u) {
      const int flat = tid + 256 * u, row = flat / VA, v = flat - row * VA;
      if (TLA % 256 && flat >= TLA) break;
      const int k0 = v * E / PA;
#pragma unroll
      for (int e = 0; e < E; ++e) As[e % PA][row * SK + k0 + e / PA] = vget<T>(ra[u], e);
    }
#pragma unroll
    for (int u = 0; u < NLB; ++u) {
      const int flat = tid + 256 * u, r = flat / VBr, v = flat - r * VBr;
      if (TLB % 256 && flat >= TLB) break;
      const int c0 = v * E / PB;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if constexpr (BT) Bs[e % PB][r * SK + c0 + e / PB] = vget<T>(rb[u], e);
        else Bs[e % PB][r * SN + c0 + e / PB] = vget<T>(rb[u], e);
      }
    }
  };

  Acc acc_r[WM][WN], acc_i[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) { acc_r[i][j][r] = 0; acc_i[i][j][r] = 0; }

  const int c16 = lane & 15, kq = lane >> 4;
  if (kbeg < kend) fetch(kbeg);
  for (int kb = kbeg; kb < kend; kb += BKt) {
    __syncthreads();                 // the previous chunk's fragments have been read
    stash();
    __syncthreads();
    if (kb + BKt < kend) fetch(kb + BKt);   // in flight while this chunk is multiplied
#pragma unroll
    for (int ks = 0; ks < BKt; ks += 4) {
      const int kk = ks + kq;
      T ar[WM], ai[WM], br[WN], bi[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const int row = wm * 16 * WM + i * 16 + c16;
        ar[i] = As[0][row * SK + kk];
        if constexpr (CA) ai[i] = As[1][row * SK + kk];
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int col = wn * 16 * WN + j * 16 + c16;
        const int bi_ = BT ? col * SK + kk : kk * SN + col;
        br[j] = Bs[0][bi_];
        if constexpr (CB) bi[j] = Bs[1][bi_];
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) M::mma(acc_r[i][j], ar[i], br[j]);
      if constexpr (CA && CB) {
#pragma unroll
        for (int i = 0; i < WM; ++i) {
          const T nai = -ai[i];
#pragma unroll
          for (int j = 0; j < WN; ++j) M::mma(acc_r[i][j], nai, bi[j]);
        }
      }
      if constexpr (CB) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) M::mma(acc_i[i][j], ar[i], bi[j]);
      }
      if constexpr (CA) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) M::mma(acc_i[i][j], ai[i], br[j]);
      }
    }
  }

  if (ksplit > 1) {
    T* w = ws + ((long)blockIdx.z * g.m * g.n) * 2;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = m0 + wm * 16 * WM + i * 16 + M::row(lane, r);
          const int gj = n0 + wn * 16 * WN + j * 16 + c16;
          if (gi < g.m && gj < g.n) {
            w[2 * ((long)gi * g.n + gj)] = acc_r[i][j][r];
            w[2 * ((long)gi * g.n + gj) + 1] = CPLX ? acc_i[i][j][r] : T(0);
          }
        }
    return;
  }
  T* C0 = g.C ? g.C + b * g.sC * (g.cC ? 2 : 1) : nullptr;
  double2* D0 = g.D ? g.D + b * g.sD : nullptr;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm * 16 * WM + i * 16 + M::row(lane, r);
        int gj = n0 + wn * 16 * WN + j * 16 + c16;
        if (gi >= g.m || gj >= g.n) continue;
        T* C = C0;
        double2* D = D0;
        if (g.vn) {           // virtual columns: member gj / vn
          const int mb = gj / g.vn;
          gj -= mb * g.vn;
          if (C) C += (long)mb * g.sC * (g.cC ? 2 : 1);
          if (D) D += (long)mb * g.sD;
        }
        const double xr = (double)acc_r[i][j][r], xi = CPLX ? (double)acc_i[i][j][r] : 0.0;
        double vr = g.ar * xr - g.ai * xi;
        double vi = g.ar * xi + g.ai * xr;
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

// split-k workspace, one per (stream, element type), grown on demand. Streams
// that run concurrently (the branches of a batch) therefore never share one.
// Entries live until gemm_release_workspace(stream) or the process ends (never
// freed during static destruction, so no device call runs then).
struct WsKey {
  hipStream_t st;
  int tsz;
  bool operator<(const WsKey& o) const { return st != o.st ? st < o.st : tsz < o.tsz; }
};
std::mutex& ws_mutex() {
  static std::mutex* m = new std::mutex();
  return *m;
}
std::map<WsKey, DevBuf*>& ws_map() {
  static auto* m = new std::map<WsKey, DevBuf*>();
  return *m;
}
DevBuf& workspace(hipStream_t st, int tsz) {
  std::lock_guard<std::mutex> lk(ws_mutex());
  DevBuf*& b = ws_map()[WsKey{st, tsz}];
  if (!b) b = new DevBuf();
  return *b;
}

}  // namespace

template <typename T> GemmArgs<T> gemm_args() {
  GemmArgs<T> g{};
  g.batch = 1;
  g.ar = 1.0;
  g.opA = g.opB = OP_N;
  return g;
}

// launch of the tiled kernel for one (WM, WN) configuration
template <typename T, bool CA, bool CB, bool BT, int WM, int WN>
void launch_tile(const GemmArgs<T>& g, dim3 grid, int ksplit, int kchunk, T* ws, hipStream_t st) {
  hipLaunchKernelGGL((gemm_tile_kernel<T, CA, CB, BT, WM, WN>), grid, dim3(256), 0, st, g, ksplit, kchunk, ws);
}

template <typename T, bool CA, bool CB, bool BT>
void launch_tile_cfg(const GemmArgs<T>& g, int cfg, dim3 grid, int ksplit, int kchunk, T* ws, hipStream_t st) {
  switch (cfg) {
    case 0: launch_tile<T, CA, CB, BT, 2, 2>(g, grid, ksplit, kchunk, ws, st); break;
    case 1: launch_tile<T, CA, CB, BT, 2, 4>(g, grid, ksplit, kchunk, ws, st); break;
    case 2: launch_tile<T, CA, CB, BT, 4, 2>(g, grid, ksplit, kchunk, ws, st); break;
    case 4: launch_tile<T, CA, CB, BT, 1, 2>(g, grid, ksplit, kchunk, ws, st); break;
    case 5: launch_tile<T, CA, CB, BT, 1, 4>(g, grid, ksplit, kchunk, ws, st); break;
    default:
      if constexpr (sizeof(T) == 4) launch_tile<T, CA, CB, BT, 4, 4>(g, grid, ksplit, kchunk, ws, st);
      break;   // not chosen for double (tile_config)
  }
}

// (WM, WN) of the tile configurations; the 32-row ones serve only m <= 32
// (products with few rows, such as those of systems with few electrons)
constexpr int kNumTileCfg = 6;
constexpr int kTileWM[kNumTileCfg] = {2, 2, 4, 4, 1, 1}, kTileWN[kNumTileCfg] = {2, 4, 2, 4, 2, 4};

// the tiled kernel applies: A untransposed (k contiguous), B untransposed or
// transposed, no conjugation, 16-byte aligned rows and bases
template <typename T> bool tile_applies(const GemmArgs<T>& g) {
  if (g.opA != OP_N || (g.opB != OP_N && g.opB != OP_T)) return false;
  const long pa = g.cA ? 2 : 1, pb = g.cB ? 2 : 1, sz = sizeof(T);
  const auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (!al(g.A) || !al(g.B)) return false;
  if ((g.lda * pa * sz) % 16 || (g.ldb * pb * sz) % 16) return false;
  if (g.batch > 1 && ((g.sA * pa * sz) % 16 || (g.sB * pb * sz) % 16)) return false;
  return g.m >= 32 && g.n >= 32 && g.k >= 16;
}

// tile configuration with the least padded work; double precision stops at
// 128 x 64 (its accumulators take twice the registers)
template <typename T> int tile_config(const GemmArgs<T>& g) {
  int best = -1;
  long best_area = 0;
  for (int c = 0; c < kNumTileCfg; ++c) {
    if (sizeof(T) == 8 && c == 3) continue;
    if (kTileWM[c] == 1 && g.m > 32) continue;   // 32-row tiles reuse operands half as often
    const long bm = 32 * kTileWM[c], bn = 32 * kTileWN[c];
    const long area = ceil_div(g.m, (int)bm) * bm * ceil_div(g.n, (int)bn) * bn;
    if (best < 0 || area < best_area || (area == best_area && bm * bn > 32L * kTileWM[best] * 32 * kTileWN[best])) {
      best = c;
      best_area = area;
    }
  }
  return best;
}

template <typename T> int gemm(const GemmArgs<T>& g, hipStream_t st) {
  AFQ_CHECK(g.m >= 0 && g.n >= 0 && g.k >= 0 && g.batch >= 0, AFQ_E_INVALID, "gemm: negative size");
  if (g.m == 0 || g.n == 0 || g.batch == 0) return AFQ_OK;
  AFQ_CHECK(g.A && g.B && (g.C || g.D), AFQ_E_INVALID, "gemm: null operand");
  if (g.vn) {
    // virtual columns need the tiled kernel with B k-major, whole vectors per
    // member and no split of k; otherwise run the members as a batch
    AFQ_CHECK(g.vn > 0 && g.batch == 1 && g.n % g.vn == 0, AFQ_E_INVALID, "gemm: bad virtual column count");
    const int vec = (int)(16 / sizeof(T)) / (g.cB ? 2 : 1);
    const long tiles = (long)ceil_div(g.m, 64) * ceil_div(g.n, 128);
    const bool ok = g.opB == OP_N && g.vn % vec == 0 && tile_applies(g) &&
                    !(tiles < 512 && g.k / 2 >= 1024) && (g.sB * (g.cB ? 2 : 1) * (long)sizeof(T)) % 16 == 0;
    if (!ok) {
      GemmArgs<T> b = g;
      b.batch = g.n / g.vn;
      b.n = g.vn;
      b.vn = 0;
      return gemm<T>(b, st);
    }
  }
  const bool tiled = tile_applies(g);
  const int cfg = tiled ? tile_config(g) : -1;
  const int bm = tiled ? 32 * kTileWM[cfg] : BM, bn = tiled ? 32 * kTileWN[cfg] : BN;
  const int tiles_m = ceil_div(g.m, bm), tiles_n = ceil_div(g.n, bn);
  AFQ_CHECK(tiles_m <= 65535, AFQ_E_INVALID, "gemm: m too large");
  // split k when few output tiles share a long contraction
  int ksplit = 1;
  const long tiles = (long)tiles_m * tiles_n * g.batch;
  while (!g.vn && tiles * ksplit < 512 && g.k / (ksplit * 2) >= 1024 && ksplit < 64) ksplit *= 2;
  const int kchunk = round_up(ceil_div(g.k, ksplit), BK);
  AFQ_CHECK((long)g.batch * ksplit <= 65535, AFQ_E_INVALID, "gemm: batch too large");
  T* ws = nullptr;
  if (ksplit > 1) {
    const size_t need = (size_t)g.batch * ksplit * g.m * g.n * 2 * sizeof(T);
    DevBuf& w = workspace(st, (int)sizeof(T));
    if (w.bytes < need) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      AFQ_TRY_HIP(hipStreamIsCapturing(st, &cs));
      AFQ_CHECK(cs == hipStreamCaptureStatusNone, AFQ_E_STATE,
                "gemm: split-k workspace must be sized by an eager call before graph capture");
      AFQ_TRY_HIP(hipStreamSynchronize(st));   // the old workspace may still be in use
      AFQ_RET(w.alloc(need));
    }
    ws = w.as<T>();
  }
  dim3 grid(tiles_n, tiles_m, g.batch * ksplit);
  if (tiled) {
    const bool bt = g.opB == OP_T;
#define AFQ_TILE(CA_, CB_)                                                             \
  (bt ? launch_tile_cfg<T, CA_, CB_, true>(g, cfg, grid, ksplit, kchunk, ws, st)       \
      : launch_tile_cfg<T, CA_, CB_, false>(g, cfg, grid, ksplit, kchunk, ws, st))
    if (g.cA && g.cB) AFQ_TILE(true, true);
    else if (g.cA) AFQ_TILE(true, false);
    else if (g.cB) AFQ_TILE(false, true);
    else AFQ_TILE(false, false);
#undef AFQ_TILE
  } else if (g.cA && g.cB) {
    hipLaunchKernelGGL((gemm_mfma_kernel<T, true, true>), grid, dim3(256), 0, st, g, ksplit, kchunk, ws);
  } else if (g.cA) {
    hipLaunchKernelGGL((gemm_mfma_kernel<T, true, false>), grid, dim3(256), 0, st, g, ksplit, kchunk, ws);
  } else if (g.cB) {
    hipLaunchKernelGGL((gemm_mfma_kernel<T, false, true>), grid, dim3(256), 0, st, g, ksplit, kchunk, ws);
  } else {
    hipLaunchKernelGGL((gemm_mfma_kernel<T, false, false>), grid, dim3(256), 0, st, g, ksplit, kchunk, ws);
  }
  AFQ_TRY_HIP(hipGetLastError());
  if (ksplit > 1) {
    const long total = (long)g.m * g.n * g.batch;
    const int blocks = (int)std::min<long>(ceil_div(total, 256), 65536);
    hipLaunchKernelGGL(gemm_splitk_reduce<T>, dim3(blocks), dim3(256), 0, st, g, ksplit, ws);
    AFQ_TRY_HIP(hipGetLastError());
  }
  return AFQ_OK;
}

void gemm_release_workspace(hipStream_t st) {
  std::lock_guard<std::mutex> lk(ws_mutex());
  for (int tsz : {4, 8}) {
    auto it = ws_map().find(WsKey{st, tsz});
    if (it == ws_map().end()) continue;
    (void)hipStreamSynchronize(st);
    delete it->second;
    ws_map().erase(it);
  }
}

template int gemm<double>(const GemmArgs<double>&, hipStream_t);
template int gemm<float>(const GemmArgs<float>&, hipStream_t);
template GemmArgs<double> gemm_args<double>();
template GemmArgs<float> gemm_args<float>();
