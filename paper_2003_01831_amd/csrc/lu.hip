// Batched small dense FP64 factorisations, one workgroup per matrix with the
// matrix held in registers (element e = tid + NT*j of the row-major n x n
// matrix lives in thread tid, slot j):
//   * Gauss-Jordan inverse with partial pivoting and log-determinant (overlap
//     matrices S = T^H W: Theta = W S^-1, log O = log det S);
//   * Cholesky factor R of a Hermitian Gram matrix W^H W and its inverse, for
//     CholeskyQR (Q = W R^-1, det R > 0).
// Pivot rows are tracked implicitly (no physical swaps); the pivot row and
// column are broadcast through LDS, two barriers per elimination step.
#include "common.h"

namespace {

constexpr int NMAX = 128;

template <int NT>
struct GjShared {
  double2 rowp[NMAX], colk[NMAX];
  double2 pivs[NMAX];
  int used[NMAX], perm[NMAX], q[NMAX];
  double red_v[NT / 64];
  int red_i[NT / 64];
  double2 red_z[NT / 64];
  double2 red_l[NT / 64];
  int p, sing;
  double d;
};

// Row and column of register slot j (element e = tid + NT j) without an
// integer division: r = mulhi(e, m) with m = ceil(2^32 / n) is exact for the
// e < 2^16, 2 <= n <= 128 used here; for n = 1 (m = 2^32 does not fit in 32
// bits) r = e. Rows of empty slots (e >= n^2) are >= n.
struct SlotMap {
  unsigned m;
  int n;
  __device__ explicit SlotMap(int n_)
      : m(n_ > 1 ? (unsigned)((0x100000000ull + (unsigned)n_ - 1) / (unsigned)n_) : 0u), n(n_) {}
  __device__ int row(int e) const { return n > 1 ? (int)__umulhi((unsigned)e, m) : e; }
  __device__ int col(int e, int r) const { return e - r * n; }
};

// Gauss-Jordan inverse without pivoting (pivot row k at step k) on the
// register-resident matrix, for the triangular factor of CholeskyQR (its
// diagonal is positive; a zero or non-finite pivot flags the matrix singular
// and is taken as 1). Two barriers per step: the pivot row and column are
// broadcast through LDS, then every element is updated.
template <int NT, int EPT>
__device__ void gj_unpivoted(double2 (&a)[EPT], int n, GjShared<NT>& sh) {
  const int tid = threadIdx.x;
  const SlotMap sm(n);
  for (int k = 0; k < n; ++k) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + NT * j, r = sm.row(e), c = sm.col(e, r);
      if (r < n) {
        if (r == k) sh.rowp[c] = a[j];
        if (c == k) sh.colk[r] = a[j];
      }
    }
    __syncthreads();
    double2 piv = sh.rowp[k];
    const double pm = cabs2(piv);
    if (!(pm > 0.0) || !isfinite(pm)) {
      if (tid == 0) sh.sing = 1;
      piv = make_double2(1.0, 0.0);
    }
    const double2 ipiv = cdiv(make_double2(1.0, 0.0), piv);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + NT * j, r = sm.row(e), c = sm.col(e, r);
      if (r < n) {
        const double2 rp = c == k ? ipiv : cmul(sh.rowp[c], ipiv);
        if (r == k) {
          a[j] = rp;
        } else {
          const double2 base = c == k ? make_double2(0.0, 0.0) : a[j];
          a[j] = csub(base, cmul(sh.colk[r], rp));
        }
      }
    }
    __syncthreads();
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
// One elimination step, pivot column k = k0 + KC of column group k0 / CB: the
// column's place KC in the register block is a compile-time constant (a
// runtime one would make the block a memory-resident array)
template <int NT, int RB, int CB, int KC>
__device__ __forceinline__ void gj_step(double2 (&a)[RB][CB], int k0, int n, int nrg, int rg, int cg, bool act,
                                        unsigned long long& used0, unsigned long long& used1, GjShared<NT>& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = k0 + KC, cgk = k0 / CB;
  // 1. candidates of column k: waves overlapping threads [cgk nrg, (cgk + 1) nrg)
  const int t0 = cgk * nrg, t1 = t0 + nrg - 1;
  const int w0 = t0 >> 6, w1 = t1 >> 6;
  if (wave >= w0 && wave <= w1) {
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
  int bi = sh.red_i[0];
  double2 bv = sh.red_z[0];
  if (w1 > w0 && (sh.red_v[1] > best || (sh.red_v[1] == best && sh.red_i[1] < bi))) {
    best = sh.red_v[1];
    bi = sh.red_i[1];
    bv = sh.red_z[1];
  }
  bool bad = false;
  if (bi < 0 || bi >= n) {   // no usable candidate (a non-finite column): first unused row
    bad = true;
    bi = ~used0 ? __ffsll((long long)~used0) - 1 : 64 + __ffsll((long long)~used1) - 1;
    if (bi >= n) bi = n - 1;
  }
  const int p = bi;
  if (p < 64) used0 |= 1ull << p;
  else used1 |= 1ull << (p - 64);
  double2 piv = bv;
  const double pm = cabs2(piv);
  if (bad || !(pm > 0.0) || !isfinite(pm)) {
    bad = true;
    piv = make_double2(1.0, 0.0);
  }
  const double2 ipiv = cdiv(make_double2(1.0, 0.0), piv);
  if (tid == 0) {
    sh.pivs[k] = piv;
    sh.perm[k] = p;
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
  if (act && cg == cgk) {
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int r = rg * RB + i;
      if (r < n) sh.colk[r] = a[i][KC];
      a[i][KC] = make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  // 3. update; the pivot row becomes the scaled row
  if (act) {
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const double2 ck = sh.colk[rg * RB + i];
#pragma unroll
      for (int c = 0; c < CB; ++c) a[i][c] = csub(a[i][c], cmul(ck, sh.rowp[cg * CB + c]));
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

template <int NT, int RB, int CB, int KC = 0>
__device__ __forceinline__ void gj_group(double2 (&a)[RB][CB], int k0, int n, int nrg, int rg, int cg, bool act,
                                         unsigned long long& used0, unsigned long long& used1, GjShared<NT>& sh) {
  if constexpr (KC < CB) {
    if (k0 + KC < n) {
      gj_step<NT, RB, CB, KC>(a, k0, n, nrg, rg, cg, act, used0, used1, sh);
      gj_group<NT, RB, CB, KC + 1>(a, k0, n, nrg, rg, cg, act, used0, used1, sh);
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
template <int NT, int RB, int CB>
__device__ void gj_blocked(double2 (&a)[RB][CB], int n, int nrg, int rg, int cg, bool act, GjShared<NT>& sh) {
  unsigned long long used0 = 0, used1 = 0;   // rows already taken as pivots (n <= 128)
  for (int k0 = 0; k0 < n; k0 += CB) gj_group<NT, RB, CB>(a, k0, n, nrg, rg, cg, act, used0, used1, sh);
  __syncthreads();
}

template <int NT, int RB, int CB, bool FULL>
__device__ void gj_body(const double2* __restrict__ S, long stride, int n,
                                                double2* __restrict__ inv, double2* __restrict__ logdet,
                                                long ld_logdet, int* __restrict__ sing, long ld_sing) {
  __shared__ GjShared<NT> sh;
  const long b = blockIdx.x;
  const int tid = threadIdx.x;
  const int nrg = (n + RB - 1) / RB, ncg = (n + CB - 1) / CB;
  const int cg = tid / nrg, rg = tid - cg * nrg;
  const bool act = cg < ncg;
  double2 a[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int r = rg * RB + i, cc = cg * CB + c;
      a[i][c] = act && r < n && cc < n ? S[b * stride + (long)r * n + cc] : make_double2(0.0, 0.0);
    }
  // broadcast entries beyond n stay zero, so the padding of the blocks does too
  for (int e = tid; e < NMAX; e += NT) {
    sh.rowp[e] = make_double2(0.0, 0.0);
    sh.colk[e] = make_double2(0.0, 0.0);
  }
  if (tid == 0) sh.sing = 0;
  __syncthreads();
  gj_blocked<NT, RB, CB>(a, n, nrg, rg, cg, act, sh);
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

template <int NT, int EPT>
__global__ __launch_bounds__(NT) void chol_inv_kernel(const double2* __restrict__ G, long stride, int n,
                                                      double2* __restrict__ rinv, double2* __restrict__ logdet,
                                                      long ld_logdet, int* __restrict__ sing, long ld_sing) {
  __shared__ GjShared<NT> sh;
  const long b = blockIdx.x;
  const int tid = threadIdx.x, nn = n * n;
  double2 a[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = tid + NT * j;
    a[j] = e < nn ? G[b * stride + e] : make_double2(0.0, 0.0);
  }
  if (tid == 0) sh.sing = 0;
  __syncthreads();
  const SlotMap sm(n);
  double ldr = 0.0;
  // right-looking Cholesky G = R^H R on the upper triangle
  for (int k = 0; k < n; ++k) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + NT * j;
      if (e == k * n + k) {
        double d = sqrt(a[j].x);
        if (!(d > 0.0) || !isfinite(d)) { sh.sing = 1; d = 1.0; }
        sh.d = d;
      }
    }
    __syncthreads();
    const double d = sh.d, id = 1.0 / d;
    if (tid == 0) ldr += log(d);   // only thread 0 reports it
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + NT * j, r = sm.row(e), c = sm.col(e, r);
      if (r == k && c >= k) {
        a[j] = c == k ? make_double2(d, 0.0) : cscale(a[j], id);
        sh.rowp[c] = a[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + NT * j, r = sm.row(e), c = sm.col(e, r);
      if (r > k && r < n && c >= r) a[j] = csub(a[j], cmul(cconj(sh.rowp[r]), sh.rowp[c]));
    }
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = tid + NT * j, r = sm.row(e);
    if (r < n && r > sm.col(e, r)) a[j] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  gj_unpivoted<NT, EPT>(a, n, sh);
  if (tid == 0) {
    logdet[b * ld_logdet] = make_double2(ldr, 0.0);
    sing[b * ld_sing] = sh.sing;
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = tid + NT * j;
    if (e < nn) rinv[b * stride + e] = a[j];
  }
}

// Gauss-Jordan inverse + log det, and log det only (the same elimination,
// whose pivots are those of LU with partial pivoting)
// two workgroups per CU: at most 128 VGPRs for 512 threads
template <int NT, int RB, int CB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void gj_kernel_full(const double2* S, long stride, int n, double2* inv,
                                                     double2* logdet, long ld_logdet, int* sing, long ld_sing) {
  gj_body<NT, RB, CB, true>(S, stride, n, inv, logdet, ld_logdet, sing, ld_sing);
}
template <int NT, int RB, int CB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void gj_kernel_det(const double2* S, long stride, int n, double2* inv,
                                                    double2* logdet, long ld_logdet, int* sing, long ld_sing) {
  gj_body<NT, RB, CB, false>(S, stride, n, inv, logdet, ld_logdet, sing, ld_sing);
}
}  // namespace

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

#define AFQ_SMALL_DISPATCH(KERNEL, ...)                                                    \
  do {                                                                                     \
    if (n <= 32)                                                                           \
      hipLaunchKernelGGL((KERNEL<256, 4>), dim3(batch), dim3(256), 0, st, __VA_ARGS__);    \
    else if (n <= 64)                                                                      \
      hipLaunchKernelGGL((KERNEL<256, 16>), dim3(batch), dim3(256), 0, st, __VA_ARGS__);   \
    else if (n <= 101)                                                                     \
      hipLaunchKernelGGL((KERNEL<512, 20>), dim3(batch), dim3(512), 0, st, __VA_ARGS__);   \
    else                                                                                   \
      hipLaunchKernelGGL((KERNEL<1024, 16>), dim3(batch), dim3(1024), 0, st, __VA_ARGS__); \
  } while (0)

int lu_inverse(const double2* S, long stride, int n, int batch, double2* inv, double2* logdet,
               long ld_logdet, int* sing, long ld_sing, hipStream_t st) {
  AFQ_CHECK(n >= 1 && n <= NMAX, AFQ_E_UNSUPPORTED, "lu_inverse: n must be in [1, 128]");
  AFQ_CHECK(stride >= (long)n * n, AFQ_E_INVALID, "lu_inverse: stride < n*n");
  if (batch <= 0) return AFQ_OK;
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
  AFQ_SMALL_DISPATCH(chol_inv_kernel, G, stride, n, rinv, logdet, ld_logdet, sing, ld_sing);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
