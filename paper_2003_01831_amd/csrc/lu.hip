// Batched small dense FP64 factorisations, one workgroup per matrix with the
// matrix held in registers, thread t owning a fixed RB x CB block:
//   * Gauss-Jordan inverse with partial pivoting and log-determinant (overlap
//     matrices S = T^H W: Theta = W S^-1, log O = log det S);
//   * Cholesky factor R of a Hermitian Gram matrix W^H W and its inverse, for
//     CholeskyQR (Q = W R^-1, det R > 0).
// Pivot rows are tracked implicitly (no physical swaps); the pivot row and
// column are broadcast through LDS, two barriers per elimination step.
#include "common.h"

namespace {

constexpr int NMAX = 128;

// z - x y in four fused multiply-adds
__device__ __forceinline__ double2 cfnma(double2 x, double2 y, double2 z) {
  const double re = fma(x.y, y.y, fma(-x.x, y.x, z.x));
  const double im = fma(-x.y, y.x, fma(-x.x, y.y, z.y));
  return make_double2(re, im);
}

// 1 / p = conj(p) / |p|^2 with one division: p is first scaled by the power
// of two that brings its larger part into [1, 2), so |p|^2 neither overflows
// nor underflows (p != 0, finite)
__device__ __forceinline__ double2 crecip(double2 p) {
  const int e = ilogb(fmax(fabs(p.x), fabs(p.y)));
  const double sx = ldexp(p.x, -e), sy = ldexp(p.y, -e);
  const double inv = 1.0 / fma(sx, sx, sy * sy);
  return make_double2(ldexp(sx * inv, -e), ldexp(-sy * inv, -e));
}

template <int NT>
struct GjShared {
  double2 rowp[NMAX], colk[NMAX];
  double2 pivs[NMAX];
  int used[NMAX], perm[NMAX], q[NMAX];
  double red_v[NT / 64];
  int red_i[NT / 64];
  double2 red_z[NT / 64];
  double2 red_l[NT / 64];
  int sing;
};

// One elimination step, pivot column k = k0 + KC of column group k0 / CB: the
// column's place KC in the register block is a compile-time constant (a
// runtime one would make the block a memory-resident array). Without PIV the
// pivot row is k (the triangular factor of CholeskyQR, whose diagonal is
// positive; a zero or non-finite pivot flags the matrix singular and is taken
// as 1).
template <int NT, int RB, int CB, int KC, bool PIV>
__device__ __forceinline__ void gj_step(double2 (&a)[RB][CB], int k0, int n, int nrg, int rg, int cg, bool act,
                                        unsigned long long& used0, unsigned long long& used1, GjShared<NT>& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = k0 + KC, cgk = k0 / CB;
  // 1. candidates of column k: waves overlapping threads [cgk nrg, (cgk + 1) nrg)
  const int t0 = cgk * nrg, t1 = t0 + nrg - 1;
  const int w0 = t0 >> 6, w1 = t1 >> 6;
  if constexpr (!PIV) {   // the holder of (k, k) posts it
    const int ik = k - rg * RB;
    unsigned kb = act && cg == cgk && ik >= 0 && ik < RB ? 1u << ik : 0u;
    __asm__ volatile("" : "+v"(kb));
    if (kb) {
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if ((kb >> i) & 1) sh.red_z[0] = a[i][KC];
    }
  } else if (wave >= w0 && wave <= w1) {
    double best = -1.0;
    int bi = 1 << 30;
    double2 bv = make_double2(0.0, 0.0);
    if (act && cg == cgk) {
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int r = rg * RB + i;
        const bool used = r < 64 ? (used0 >> r) & 1 : (used1 >> (r - 64)) & 1;
        const double m = cabs2(a[i][KC]);
        if (r < n && !used && m > best) { best = m; bi = r; bv = a[i][KC]; }
      }
    }
    double rbest = best;
    int rbi = bi;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(rbest, off);
      const int oi = __shfl_xor(rbi, off);
      if (ov > rbest || (ov == rbest && oi < rbi)) { rbest = ov; rbi = oi; }
    }
    const int slot = wave - w0;
    if (lane == 0) { sh.red_v[slot] = rbest; sh.red_i[slot] = rbi; }
    if (rbi == bi && bi < n) sh.red_z[slot] = bv;
  }
  __syncthreads();
  // 2. pivot, broadcasts
  double best = sh.red_v[0];
  int bi = PIV ? sh.red_i[0] : k;
  double2 bv = sh.red_z[0];
  bool bad = false;
  if constexpr (PIV) {
    if (w1 > w0 && (sh.red_v[1] > best || (sh.red_v[1] == best && sh.red_i[1] < bi))) {
      best = sh.red_v[1];
      bi = sh.red_i[1];
      bv = sh.red_z[1];
    }
    if (bi < 0 || bi >= n) {   // no usable candidate (a non-finite column): first unused row
      bad = true;
      bi = ~used0 ? __ffsll((long long)~used0) - 1 : 64 + __ffsll((long long)~used1) - 1;
      if (bi >= n) bi = n - 1;
    }
    if (bi < 64) used0 |= 1ull << bi;
    else used1 |= 1ull << (bi - 64);
  }
  const int p = bi;
  double2 piv = bv;
  const double pm = cabs2(piv);
  if (bad || !(pm > 0.0) || !isfinite(pm)) {
    bad = true;
    piv = make_double2(1.0, 0.0);
  }
  const double2 ipiv = crecip(piv);
  if (tid == 0) {
    if constexpr (PIV) {
      sh.pivs[k] = piv;
      sh.perm[k] = p;
    }
    if (bad) sh.sing = 1;
  }
  // the row of the block that holds p, as a bit (a mask the compiler cannot
  // see through, for the same reason as KC)
  const int ip = p - rg * RB;
  unsigned pbit = act && ip >= 0 && ip < RB ? 1u << ip : 0u;
  __asm__ volatile("" : "+v"(pbit));
  if (pbit) {
#pragma unroll
    for (int i = 0; i < RB; ++i)
      if ((pbit >> i) & 1)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          const int cc = cg * CB + c;
          if (cc < n) sh.rowp[cc] = c == KC && cg == cgk ? ipiv : cmul(a[i][c], ipiv);
        }
  }
  // pivot column entry r = rg RB + i at colk[i CKS + rg]: a lane's RB entries
  // are CKS apart and neighbouring lanes' adjacent, so the 16-byte reads of
  // the update below do not conflict on banks (the plain order put the lanes
  // 64 bytes apart)
  constexpr int CKS = NMAX / RB;
  static_assert(NMAX % RB == 0, "pivot column layout");
  if (act && cg == cgk) {
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int r = rg * RB + i;
      if (r < n) sh.colk[i * CKS + rg] = a[i][KC];
      a[i][KC] = make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  // 3. update; the pivot row becomes the scaled row
  if (act) {
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const double2 ck = sh.colk[i * CKS + rg];
#pragma unroll
      for (int c = 0; c < CB; ++c) a[i][c] = cfnma(ck, sh.rowp[cg * CB + c], a[i][c]);
    }
    if (pbit) {
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if ((pbit >> i) & 1)
#pragma unroll
          for (int c = 0; c < CB; ++c) a[i][c] = sh.rowp[cg * CB + c];
    }
  }
}

template <int NT, int RB, int CB, bool PIV, int KC = 0>
__device__ __forceinline__ void gj_group(double2 (&a)[RB][CB], int k0, int n, int nrg, int rg, int cg, bool act,
                                         unsigned long long& used0, unsigned long long& used1, GjShared<NT>& sh) {
  if constexpr (KC < CB) {
    if (k0 + KC < n) {
      gj_step<NT, RB, CB, KC, PIV>(a, k0, n, nrg, rg, cg, act, used0, used1, sh);
      gj_group<NT, RB, CB, PIV, KC + 1>(a, k0, n, nrg, rg, cg, act, used0, used1, sh);
    }
  }
}

// Gauss-Jordan elimination with partial pivoting on a block layout: thread
// t holds the RB x CB block (rg, cg) of the matrix, t = cg * nrg + rg with
// nrg = ceil(n / RB) row groups, so the candidates of a pivot column sit in
// the nrg consecutive threads of its column group (one or two waves). Per
// step k, two barriers:
//   1. the lanes of column k take their best live row (largest |a|^2, then
//      lowest row), their waves reduce it and the winning lane posts row and
//      value;
//   2. every thread takes pivot row p and 1 / pivot; the lanes of row p
//      broadcast it scaled by 1 / pivot (column k: 1 / pivot), the lanes of
//      column k broadcast that column and clear it;
// then every element takes a[r][c] -= colk[r] rowp[c] with no branch, and the
// lanes of row p overwrite it with the scaled pivot row. The result is the
// in-place inverse up to the pivot permutation (no physical row swaps). The
// pivots go to sh.pivs (their logs are summed afterwards, in parallel) and
// the pivot order to sh.perm. A column without a usable pivot (zero or non-
// finite) flags the matrix singular and takes pivot 1 in the first row not
// yet used.
template <int NT, int RB, int CB, bool PIV>
__device__ void gj_blocked(double2 (&a)[RB][CB], int n, int nrg, int rg, int cg, bool act, GjShared<NT>& sh) {
  unsigned long long used0 = 0, used1 = 0;   // rows already taken as pivots (n <= 128)
  for (int k0 = 0; k0 < n; k0 += CB) gj_group<NT, RB, CB, PIV>(a, k0, n, nrg, rg, cg, act, used0, used1, sh);
  __syncthreads();
}

// The blocks of thread tid: column group cg, row group rg, active if cg < ncg;
// element (r, c) of the row-major n x n matrix at m + r n + c, zero outside.
// The broadcast arrays start zero, so entries beyond n stay zero and the
// padding of the blocks does too.
template <int NT, int RB, int CB>
__device__ void blocks_load(double2 (&a)[RB][CB], const double2* __restrict__ m, int n, int& nrg, int& rg,
                            int& cg, bool& act, GjShared<NT>& sh) {
  const int tid = threadIdx.x;
  nrg = (n + RB - 1) / RB;
  const int ncg = (n + CB - 1) / CB;
  cg = tid / nrg;
  rg = tid - cg * nrg;
  act = cg < ncg;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int r = rg * RB + i, cc = cg * CB + c;
      a[i][c] = act && r < n && cc < n ? m[(long)r * n + cc] : make_double2(0.0, 0.0);
    }
  for (int e = tid; e < NMAX; e += NT) {
    sh.rowp[e] = make_double2(0.0, 0.0);
    sh.colk[e] = make_double2(0.0, 0.0);
  }
  if (tid == 0) sh.sing = 0;
  __syncthreads();
}

// matrix b of the batch at S (stride elements apart)
template <int NT, int RB, int CB, bool FULL>
__device__ __forceinline__ void gj_body(const double2* __restrict__ S, long stride, int n,
                                                double2* __restrict__ inv, double2* __restrict__ logdet,
                                                long ld_logdet, int* __restrict__ sing, long ld_sing, long b) {
  __shared__ GjShared<NT> sh;
  const int tid = threadIdx.x;
  double2 a[RB][CB];
  int nrg, rg, cg;
  bool act;
  blocks_load<NT, RB, CB>(a, S + b * stride, n, nrg, rg, cg, act, sh);
  gj_blocked<NT, RB, CB, true>(a, n, nrg, rg, cg, act, sh);
  // log det = sum_k log(pivot_k) (+ i pi for an odd permutation): threads k < n
  // take one pivot each, waves reduce, the per-wave sums are added in order
  double2 ld = tid < n ? clog(sh.pivs[tid]) : make_double2(0.0, 0.0);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    ld.x += __shfl_xor(ld.x, off);
    ld.y += __shfl_xor(ld.y, off);
  }
  if ((tid & 63) == 0 && tid < NMAX) sh.red_l[tid >> 6] = ld;
  __syncthreads();
  if (tid == 0) {
    ld = sh.red_l[0];
    if (n > 64) ld = cadd(ld, sh.red_l[1]);
    // parity of the pivot permutation k -> perm[k]; inverse permutation q
    int parity = 0;
    for (int k = 0; k < n; ++k) { sh.q[sh.perm[k]] = k; sh.used[k] = 0; }
    for (int s0 = 0; s0 < n; ++s0) {
      if (sh.used[s0]) continue;
      int len = 0, x = s0;
      while (!sh.used[x]) { sh.used[x] = 1; x = sh.perm[x]; ++len; }
      parity ^= (len - 1) & 1;
    }
    if (parity) ld.y += 3.14159265358979323846;
    ld.y = remainder(ld.y, 2.0 * 3.14159265358979323846);
    logdet[b * ld_logdet] = sh.sing ? make_double2(-INFINITY, 0.0) : ld;
    sing[b * ld_sing] = sh.sing;
  }
  __syncthreads();
  if (FULL && act) {
    // inverse element (a, b) = M[perm[a]][q[b]]: the holder of M[r][c] writes (q[r], perm[c])
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int r = rg * RB + i, cc = cg * CB + c;
        if (r < n && cc < n) inv[b * stride + (long)sh.q[r] * n + sh.perm[cc]] = a[i][c];
      }
  }
}

// Cholesky factor R (G = R^H R, upper triangular) of a Hermitian positive
// definite Gram matrix and its inverse, on the register blocks of the
// Gauss-Jordan kernels. Right-looking: step k broadcasts row k unscaled, d =
// sqrt(G_kk), every element takes a[r][c] -= conj(row[r]) row[c] / d^2 with
// no branch (rows above k meet zero broadcast entries, the lower triangle is
// cleared afterwards) and the lanes of row k overwrite it with R[k][c] =
// row[c] / d, R[k][k] = d. A non-positive or non-finite d flags the matrix
// singular and is taken as 1. Then the unpivoted Gauss-Jordan inverse of R.
template <int NT, int RB, int CB>
__global__ __launch_bounds__(NT) void chol_inv_kernel(
    const double2* __restrict__ G, long stride, int n, double2* __restrict__ rinv, double2* __restrict__ logdet,
    long ld_logdet, int* __restrict__ sing, long ld_sing) {
  __shared__ GjShared<NT> sh;
  const long b = blockIdx.x;
  const int tid = threadIdx.x;
  double2 a[RB][CB];
  int nrg, rg, cg;
  bool act;
  blocks_load<NT, RB, CB>(a, G + b * stride, n, nrg, rg, cg, act, sh);
  double ldr = 0.0;   // thread 0 sums log d in step order
  for (int k = 0; k < n; ++k) {
    const int ik = k - rg * RB;
    unsigned kbit = act && ik >= 0 && ik < RB ? 1u << ik : 0u;
    __asm__ volatile("" : "+v"(kbit));
    if (kbit) {
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if ((kbit >> i) & 1)
#pragma unroll
          for (int c = 0; c < CB; ++c) {
            const int cc = cg * CB + c;
            if (cc < n) sh.rowp[cc] = cc >= k ? a[i][c] : make_double2(0.0, 0.0);
          }
    }
    __syncthreads();
    double d = sqrt(sh.rowp[k].x);
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) sh.sing = 1;
      d = 1.0;
    }
    if (tid == 0) ldr += log(d);
    const double id = 1.0 / d, id2 = id * id;
    if (act) {
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const double2 ck = cscale(cconj(sh.rowp[rg * RB + i]), id2);
#pragma unroll
        for (int c = 0; c < CB; ++c) a[i][c] = cfnma(ck, sh.rowp[cg * CB + c], a[i][c]);
      }
      if (kbit) {
#pragma unroll
        for (int i = 0; i < RB; ++i)
          if ((kbit >> i) & 1)
#pragma unroll
            for (int c = 0; c < CB; ++c) {
              const int cc = cg * CB + c;
              a[i][c] = cc == k ? make_double2(d, 0.0) : cscale(sh.rowp[cc], id);
            }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int c = 0; c < CB; ++c)
      if (rg * RB + i > cg * CB + c) a[i][c] = make_double2(0.0, 0.0);
  gj_blocked<NT, RB, CB, false>(a, n, nrg, rg, cg, act, sh);
  if (tid == 0) {
    logdet[b * ld_logdet] = make_double2(ldr, 0.0);
    sing[b * ld_sing] = sh.sing;
  }
  if (act) {
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int r = rg * RB + i, cc = cg * CB + c;
        if (r < n && cc < n) rinv[b * stride + (long)r * n + cc] = a[i][c];
      }
  }
}

// Gauss-Jordan inverse + log det, and log det only (the same elimination,
// whose pivots are those of LU with partial pivoting)
// two workgroups per CU: at most 128 VGPRs for 512 threads
template <int NT, int RB, int CB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void gj_kernel_full(const double2* S, long stride, int n, double2* inv,
                                                     double2* logdet, long ld_logdet, int* sing, long ld_sing) {
  gj_body<NT, RB, CB, true>(S, stride, n, inv, logdet, ld_logdet, sing, ld_sing, blockIdx.x);
}
template <int NT, int RB, int CB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void gj_kernel_det(const double2* S, long stride, int n, double2* inv,
                                                    double2* logdet, long ld_logdet, int* sing, long ld_sing) {
  gj_body<NT, RB, CB, false>(S, stride, n, inv, logdet, ld_logdet, sing, ld_sing, blockIdx.x);
}

// Work table of a grouped launch: the batches of up to GJ_GROUP tasks (other
// systems, both spins) of one register-block layout, passed by value (so a
// captured graph holds it); workgroup x runs matrix x - first[t] of the task t
// with first[t] <= x < first[t + 1].
constexpr int GJ_GROUP = 40;
struct GjGroupArgs {
  const double2* S[GJ_GROUP];
  double2* inv[GJ_GROUP];
  double2* logdet[GJ_GROUP];
  int* sing[GJ_GROUP];
  int stride[GJ_GROUP], n[GJ_GROUP], ld_logdet[GJ_GROUP], ld_sing[GJ_GROUP];
  int first[GJ_GROUP + 1];
  int ntask;
};

template <int NT, int RB, int CB, bool FULL>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void gj_grouped_kernel(GjGroupArgs g) {
  const int x = blockIdx.x;
  int t = 0;
  while (t + 1 < g.ntask && x >= g.first[t + 1]) ++t;
  gj_body<NT, RB, CB, FULL>(g.S[t], g.stride[t], g.n[t], g.inv[t], g.logdet[t], g.ld_logdet[t], g.sing[t],
                            g.ld_sing[t], x - g.first[t]);
}

// register-block layout of an order-n matrix (the dispatch below)
int gj_bucket(int n) { return n <= 32 ? 0 : n <= 64 ? 1 : n <= 100 ? 2 : 3; }

thread_local std::vector<GjTask>* t_gj_sink = nullptr;
}  // namespace

void lu_defer(std::vector<GjTask>* sink) { t_gj_sink = sink; }

// the tasks as few launches as possible: one per (layout, inverse or not) and
// GJ_GROUP tasks, each workgroup one matrix
int lu_inverse_grouped(const std::vector<GjTask>& tasks, hipStream_t st) {
  for (int bucket = 0; bucket < 4; ++bucket)
    for (int full = 0; full < 2; ++full) {
      GjGroupArgs g{};
      int blocks = 0;
      auto flush = [&]() -> int {
        if (g.ntask == 0) return AFQ_OK;
        g.first[g.ntask] = blocks;
#define AFQ_GJG(NT_, RB_, CB_)                                                                       \
  do {                                                                                               \
    if (full) hipLaunchKernelGGL((gj_grouped_kernel<NT_, RB_, CB_, true>), dim3(blocks), dim3(NT_), 0, st, g); \
    else hipLaunchKernelGGL((gj_grouped_kernel<NT_, RB_, CB_, false>), dim3(blocks), dim3(NT_), 0, st, g);     \
  } while (0)
        if (bucket == 0) AFQ_GJG(256, 2, 2);
        else if (bucket == 1) AFQ_GJG(256, 4, 4);
        else if (bucket == 2) AFQ_GJG(512, 4, 5);
        else AFQ_GJG(1024, 4, 4);
#undef AFQ_GJG
        AFQ_TRY_HIP(hipGetLastError());
        g = GjGroupArgs{};
        blocks = 0;
        return AFQ_OK;
      };
      for (const GjTask& k : tasks) {
        if (gj_bucket(k.n) != bucket || (k.inv != nullptr) != (full != 0) || k.batch <= 0) continue;
        const int t = g.ntask++;
        g.S[t] = k.S; g.inv[t] = k.inv; g.logdet[t] = k.logdet; g.sing[t] = k.sing;
        g.stride[t] = k.stride; g.n[t] = k.n; g.ld_logdet[t] = k.ld_logdet; g.ld_sing[t] = k.ld_sing;
        g.first[t] = blocks;
        blocks += k.batch;
        if (g.ntask == GJ_GROUP) AFQ_RET(flush());
      }
      AFQ_RET(flush());
    }
  return AFQ_OK;
}

// thread blocks: ceil(n / RB) * ceil(n / CB) <= NT
#define AFQ_GJ_DISPATCH(KERNEL, ...)                                                          \
  do {                                                                                        \
    if (n <= 32)                                                                              \
      hipLaunchKernelGGL((KERNEL<256, 2, 2>), dim3(batch), dim3(256), 0, st, __VA_ARGS__);    \
    else if (n <= 64)                                                                         \
      hipLaunchKernelGGL((KERNEL<256, 4, 4>), dim3(batch), dim3(256), 0, st, __VA_ARGS__);    \
    else if (n <= 100)                                                                        \
      hipLaunchKernelGGL((KERNEL<512, 4, 5>), dim3(batch), dim3(512), 0, st, __VA_ARGS__);    \
    else                                                                                      \
      hipLaunchKernelGGL((KERNEL<1024, 4, 4>), dim3(batch), dim3(1024), 0, st, __VA_ARGS__);  \
  } while (0)

int lu_inverse(const double2* S, long stride, int n, int batch, double2* inv, double2* logdet,
               long ld_logdet, int* sing, long ld_sing, hipStream_t st) {
  AFQ_CHECK(n >= 1 && n <= NMAX, AFQ_E_UNSUPPORTED, "lu_inverse: n must be in [1, 128]");
  AFQ_CHECK(stride >= (long)n * n, AFQ_E_INVALID, "lu_inverse: stride < n*n");
  if (batch <= 0) return AFQ_OK;
  if (t_gj_sink) {   // deferred into a grouped launch of many systems
    AFQ_CHECK(stride <= INT32_MAX && ld_logdet <= INT32_MAX && ld_sing <= INT32_MAX, AFQ_E_INVALID,
              "lu_inverse: stride too large to defer");
    t_gj_sink->push_back(GjTask{S, inv, logdet, sing, (int)stride, n, batch, (int)ld_logdet, (int)ld_sing});
    return AFQ_OK;
  }
  if (inv) AFQ_GJ_DISPATCH(gj_kernel_full, S, stride, n, inv, logdet, ld_logdet, sing, ld_sing);
  else AFQ_GJ_DISPATCH(gj_kernel_det, S, stride, n, inv, logdet, ld_logdet, sing, ld_sing);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

int chol_inverse(const double2* G, long stride, int n, int batch, double2* rinv, double2* logdet,
                 long ld_logdet, int* sing, long ld_sing, hipStream_t st) {
  AFQ_CHECK(n >= 1 && n <= NMAX, AFQ_E_UNSUPPORTED, "chol_inverse: n must be in [1, 128]");
  AFQ_CHECK(stride >= (long)n * n, AFQ_E_INVALID, "chol_inverse: stride < n*n");
  if (batch <= 0) return AFQ_OK;
  AFQ_GJ_DISPATCH(chol_inv_kernel, G, stride, n, rinv, logdet, ld_logdet, sing, ld_sing);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
