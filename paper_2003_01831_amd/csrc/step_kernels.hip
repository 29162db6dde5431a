// Elementwise and per-walker kernels of the walker step: operand packing and
// precision splits, local-energy assembly with the force bias and the
// Hubbard-Stratonovich coefficients, the mixed-energy estimator, the phaseless
// weight update and masked walker copies, and the Philox field generator.
#include "common.h"
#include "step_kernels.h"

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the two 32x32->64-bit
// multiplications with multipliers 0xD2511F53 / 0xCD9E8D57, key bumped by the
// Weyl constants 0x9E3779B9 / 0xBB67AE85 between rounds.
// ---------------------------------------------------------------------------
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
  }
  return c;
}

// two standard normals for field pair j of walker w at step `step`
__device__ inline double2 philox_normal_pair(uint64_t seed, uint32_t sys_id, uint64_t step, int w, int j) {
  const uint4 r = philox4x32_10(make_uint4((uint32_t)j, (uint32_t)w, (uint32_t)step, sys_id),
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((uint64_t)r.y << 32) | r.x, b = ((uint64_t)r.w << 32) | r.z;
  const double u1 = ((double)(a >> 11) + 0.5) * 0x1.0p-53;
  const double u2 = (double)(b >> 11) * 0x1.0p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * 3.14159265358979323846 * u2;
  return make_double2(rad * cos(ang), rad * sin(ang));
}

__global__ void fields_kernel(uint64_t seed, uint32_t sys_id, uint64_t step0, int n_steps, int nw, int X,
                              double* out, long ld_step) {
  const int npair = (X + 1) / 2;
  const long total = (long)n_steps * nw * npair;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t % npair);
    const long rest = t / npair;
    const int w = (int)(rest % nw);
    const int k = (int)(rest / nw);
    const double2 z = philox_normal_pair(seed, sys_id, step0 + k, w, j);
    double* o = out + k * ld_step + (long)w * X;
    o[2 * j] = z.x;
    if (2 * j + 1 < X) o[2 * j + 1] = z.y;
  }
}

int launch_fields(uint64_t seed, uint32_t sys_id, uint64_t step, int nw, int X, double* out, long ld_step,
                  int n_steps, hipStream_t st) {
  const long total = (long)n_steps * nw * ((X + 1) / 2);
  if (total == 0) return AFQ_OK;
  const int blocks = (int)std::min<long>(ceil_div(total, 256), 65536);
  hipLaunchKernelGGL(fields_kernel, dim3(blocks), dim3(256), 0, st, seed, sys_id, step, n_steps, nw, X, out, ld_step);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// ---------------------------------------------------------------------------
// precision conversion: split-BF16 with round-to-nearest-even
// x -> f = fp32(x); hi = bf16(f); lo = bf16(f - hi)
// ---------------------------------------------------------------------------
__device__ inline unsigned short bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

template <int PREC> struct PackOut;
template <> struct PackOut<AFQ_FP64> {
  __device__ static void put(void* hi, void*, long i, double v) { static_cast<double*>(hi)[i] = v; }
};
template <> struct PackOut<AFQ_CFP32> {
  __device__ static void put(void* hi, void*, long i, double v) { static_cast<float*>(hi)[i] = (float)v; }
};
template <> struct PackOut<AFQ_BF16X3> {
  __device__ static void put(void* hi, void* lo, long i, double v) {
    const float f = (float)v;
    const unsigned short h = bf16_rne(f);
    static_cast<unsigned short*>(hi)[i] = h;
    static_cast<unsigned short*>(lo)[i] = bf16_rne(f - bf16_to_f(h));
  }
};

// A rows (n, a) of one spin from Lt[n][off + a][k] (ntot x M complex per n)
// element (row, k) of a packed operand with `rows` rows: row-major, or
// chunk-major in k-chunks of kcm elements
__device__ inline long pack_index(long row, int k, int kp, long rows, int kcm) {
  return kcm ? ((long)(k / kcm) * rows + row) * kcm + k % kcm : row * kp + k;
}

template <int PREC>
__global__ void pack_a_kernel(const double2* __restrict__ Lt, int X, int ntot, int M, int off, int n, int np,
                              int kp, bool real_trial, void* hi, void* lo, int pad, int kcm) {
  const long rows = (long)X * np + pad;
  const long total = rows * kp;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int k = (int)(t % kp);
    const long row = t / kp;
    const int a = (int)(row % np);
    const long nn = row / np;
    double v = 0.0;
    if (a < n && nn < X) {
      const double2* src = Lt + (nn * ntot + off + a) * (long)M;
      if (k < M) v = src[k].x;
      else if (!real_trial && k < 2 * M) v = src[k - M].y;
    }
    PackOut<PREC>::put(hi, lo, pack_index(row, k, kp, rows, kcm), v);
  }
}

// B rows (w, part, b) of one spin from thetaT[w][off + b][k]
template <int PREC>
__global__ void pack_b_kernel(const double2* __restrict__ thT, int nw, int ntot, int M, int off, int n, int np,
                              int kp, bool real_trial, void* hi, void* lo, int pad, int kcm) {
  const long rows = (long)nw * 2 * np + pad;
  const long total = rows * kp;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int k = (int)(t % kp);
    const long row = t / kp;
    const int c = (int)(row % (2 * np));
    const long w = row / (2 * np);
    const int part = c >= np, b = c - part * np;
    double v = 0.0;
    if (b < n && w < nw) {
      const double2* src = thT + (w * ntot + off + b) * (long)M;
      if (k < M) {
        const double2 x = src[k];
        v = part ? x.y : x.x;
      } else if (!real_trial && k < 2 * M) {
        const double2 x = src[k - M];
        v = part ? x.x : -x.y;
      }
    }
    PackOut<PREC>::put(hi, lo, pack_index(row, k, kp, rows, kcm), v);
  }
}

static int grid_for(long total) { return (int)std::min<long>(std::max<long>(ceil_div(total, 256), 1), 262144); }

int pack_a(int prec, const double2* Lt, int X, int ntot, int M, int off, const PackShape& ps, bool real_trial,
           void* hi, void* lo, hipStream_t st) {
  const long total = ((long)X * ps.np + ps.pad) * ps.kp;
#define AFQ_PACKA(P) hipLaunchKernelGGL(pack_a_kernel<P>, dim3(grid_for(total)), dim3(256), 0, st, Lt, X, ntot, M, off, ps.n, ps.np, ps.kp, real_trial, hi, lo, ps.pad, ps.kcm)
  if (prec == AFQ_FP64) AFQ_PACKA(AFQ_FP64); else if (prec == AFQ_CFP32) AFQ_PACKA(AFQ_CFP32); else AFQ_PACKA(AFQ_BF16X3);
#undef AFQ_PACKA
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

int pack_b(int prec, const double2* thT, int nw, int ntot, int M, int off, const PackShape& ps, bool real_trial,
           void* hi, void* lo, hipStream_t st) {
  const long total = ps.rows_b(nw) * ps.kp;
#define AFQ_PACKB(P) hipLaunchKernelGGL(pack_b_kernel<P>, dim3(grid_for(total)), dim3(256), 0, st, thT, nw, ntot, M, off, ps.n, ps.np, ps.kp, real_trial, hi, lo, ps.pad, ps.kcm)
  if (prec == AFQ_FP64) AFQ_PACKB(AFQ_FP64); else if (prec == AFQ_CFP32) AFQ_PACKB(AFQ_CFP32); else AFQ_PACKB(AFQ_BF16X3);
#undef AFQ_PACKB
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// ---------------------------------------------------------------------------
// generic conversions and copies
// ---------------------------------------------------------------------------
__global__ void d2f_kernel(const double* __restrict__ x, float* __restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = (float)x[i];
}
int convert_d2f(const double* x, float* y, long n, hipStream_t st) {
  if (n <= 0) return AFQ_OK;
  hipLaunchKernelGGL(d2f_kernel, dim3(grid_for(n)), dim3(256), 0, st, x, y, n);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
__global__ void real_part_kernel(const double2* __restrict__ z, double* __restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = z[i].x;
}
int real_part(const double2* z, double* y, long n, hipStream_t st) {
  if (n <= 0) return AFQ_OK;
  hipLaunchKernelGGL(real_part_kernel, dim3(grid_for(n)), dim3(256), 0, st, z, y, n);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
__global__ void copy_kernel(const double* __restrict__ x, double* __restrict__ y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = x[i];
}
int copy_d(const double* x, double* y, long n, hipStream_t st) {
  if (n <= 0) return AFQ_OK;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, st, x, y, n);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
__global__ void fill_kernel(double* __restrict__ y, double v, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = v;
}
int fill_d(double* y, double v, long n, hipStream_t st) {
  if (n <= 0) return AFQ_OK;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, st, y, v, n);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
__global__ void fill_i_kernel(int* __restrict__ y, int v, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = v;
}
int fill_i(int* y, int v, long n, hipStream_t st) {
  if (n <= 0) return AFQ_OK;
  hipLaunchKernelGGL(fill_i_kernel, dim3(grid_for(n)), dim3(256), 0, st, y, v, n);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
// identity into an M x M real matrix
__global__ void eye_kernel(double* __restrict__ y, int M) {
  const long n = (long)M * M;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (i / M == i % M) ? 1.0 : 0.0;
}
int fill_eye(double* y, int M, hipStream_t st) {
  hipLaunchKernelGGL(eye_kernel, dim3(grid_for((long)M * M)), dim3(256), 0, st, y, M);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// broadcast the trial to every walker: W[w] = phi
__global__ void bcast_kernel(const double2* __restrict__ phi, double2* __restrict__ W, long per, int nw) {
  const long total = per * nw;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x)
    W[i] = phi[i % per];
}
int broadcast_trial(const double2* phi, double2* W, long per, int nw, hipStream_t st) {
  hipLaunchKernelGGL(bcast_kernel, dim3(grid_for(per * nw)), dim3(256), 0, st, phi, W, per, nw);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// walker copy dst[w] = src[w] for live walkers
__global__ void masked_copy_kernel(const double2* __restrict__ src, double2* __restrict__ dst, long per,
                                   const int* __restrict__ alive, int where_alive) {
  const long w = blockIdx.y;
  if ((alive[w] != 0) != (where_alive != 0)) return;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < per; i += (long)gridDim.x * blockDim.x)
    dst[w * per + i] = src[w * per + i];
}
int masked_copy(const double2* src, double2* dst, long per, int nw, const int* alive, hipStream_t st,
                bool where_alive) {
  const int bx = (int)std::min<long>(ceil_div(per, 256), 64);
  hipLaunchKernelGGL(masked_copy_kernel, dim3(bx, nw), dim3(256), 0, st, src, dst, per, alive, where_alive ? 1 : 0);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// ---------------------------------------------------------------------------
// fixed-order block reduction of several complex partial sums (256 threads)
// ---------------------------------------------------------------------------
template <int K>
__device__ inline void block_sum(double2 (&v)[K]) {
  __shared__ double2 red[K][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < K; ++q) red[q][t] = v[q];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int q = 0; q < K; ++q) red[q][t] = cadd(red[q][t], red[q][t + s]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < K; ++q) v[q] = red[q][0];
  __syncthreads();
}

// Per-walker energy assembly (one 256-thread workgroup per walker):
//   E1 = sum_s tr(ht^s Theta^s) = sum_{c,k} ht[c][k] thetaT[w][c][k]
//   vbar_n = sum_s tro[w][s][n],  EJ = 1/2 sum_n vbar_n^2,
//   EK = -1/2 sum_{n,s} troo[w][s][n],  E_L = E_II + E1 + EJ + EK.
// With coef != NULL also the propagator coefficients c_n = i sqrt(dt) x_n - dt vbar_n
// and the importance factor sum_n x_n xbar_n - xbar_n^2/2, xbar_n = -i sqrt(dt) vbar_n,
// with x from `fields` (nw x X) or the Philox stream.
template <typename CT>
__global__ __launch_bounds__(256) void assemble_kernel(AssembleArgs a, CT* __restrict__ coef) {
  const int w = blockIdx.x, t = threadIdx.x;
  const long per = (long)a.ntot * a.M;
  const double2* th = a.thetaT + w * per;
  double2 v[5] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0),
                  make_double2(0, 0)};
  const bool given = a.parts_in != nullptr;
  if (!given) {   // E1 partial sums: four independent chains keep four loads of each operand in flight
    double2 e1[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    long e = t;
    for (; e + 768 < per; e += 1024)
#pragma unroll
      for (int u = 0; u < 4; ++u) e1[u] = cadd(e1[u], cmul(a.ht[e + 256 * u], th[e + 256 * u]));
    for (; e < per; e += 256) e1[0] = cadd(e1[0], cmul(a.ht[e], th[e]));
    v[0] = cadd(cadd(e1[0], e1[1]), cadd(e1[2], e1[3]));
  }
  const double sdt = sqrt(a.dt);
  const double2* tro0 = a.tro + (long)w * 2 * a.X;
  const double2* tro1 = tro0 + a.X;
  const double2* troo0 = a.troo + (long)w * 2 * a.X;
  const double2* troo1 = troo0 + a.X;
  const int npair = (a.X + 1) / 2;
  const uint64_t step = a.step_ptr ? *a.step_ptr + a.step_off : a.step_off;
  for (int j = t; j < npair; j += 256) {
    double xs[2] = {0.0, 0.0};
    if (coef) {
      if (a.fields) {
        xs[0] = a.fields[(long)w * a.X + 2 * j];
        if (2 * j + 1 < a.X) xs[1] = a.fields[(long)w * a.X + 2 * j + 1];
      } else {
        const double2 z = philox_normal_pair(a.seed, a.sys_id, step, w, j);
        xs[0] = z.x;
        xs[1] = z.y;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int n = 2 * j + h;
      if (n >= a.X) break;
      const double2 vb = given ? a.vbar_in[(long)w * a.X + n] : cadd(tro0[n], tro1[n]);
      if (!given) {
        v[1] = cadd(v[1], cmul(vb, vb));
        v[2] = cadd(v[2], cadd(troo0[n], troo1[n]));
      }
      if (a.vbar_out) a.vbar_out[(long)w * a.X + n] = vb;
      if (coef) {
        const double x = xs[h];
        const double mfn = a.vmf ? a.vmf[n] : 0.0;           // background c_n (0: none)
        double2 xb = make_double2(sdt * vb.y, -sdt * (vb.x - mfn));  // -i sqrt(dt) (vbar - c)
        if (a.fb_cap > 0.0) {                               // cap |xbar|, keep its phase
          const double m = sqrt(cabs2(xb));
          if (m > a.fb_cap) xb = cscale(xb, a.fb_cap / m);
        }
        const double cr = sdt * xb.y, ci = sdt * (x - xb.x);   // i sqrt(dt) (x - xbar)
        CT c;
        c.x = cr;
        c.y = ci;
        coef[(long)w * a.X + n] = c;
        const double2 xb2 = cmul(xb, xb);
        v[3] = cadd(v[3], make_double2(x * xb.x - 0.5 * xb2.x, x * xb.y - 0.5 * xb2.y));
        if (a.vmf) {   // c-number -c_n i sqrt(dt) (x - xbar) of the shifted operator, and dt/2 c_n^2
          v[3].x += -mfn * cr + 0.5 * a.dt * mfn * mfn;
          v[4].x += -mfn * ci;
        }
      }
    }
  }
  block_sum<5>(v);
  if (t == 0) {
    const double2 e1 = given ? a.parts_in[3 * w] : v[0];
    const double2 ej = given ? a.parts_in[3 * w + 1] : cscale(v[1], 0.5);
    const double2 ek = given ? a.parts_in[3 * w + 2] : cscale(v[2], -0.5);
    const double2 el = make_double2(a.e_core + e1.x + ej.x + ek.x, e1.y + ej.y + ek.y);
    a.eloc[w] = el;
    if (a.eloc_out) a.eloc_out[w] = el;
    if (a.parts) { a.parts[3 * w] = e1; a.parts[3 * w + 1] = ej; a.parts[3 * w + 2] = ek; }
    if (a.lfac) a.lfac[w] = make_double2(v[3].x, v[4].x);
  }
}

int launch_assemble(const AssembleArgs& a, void* coef, bool coef_f32, hipStream_t st) {
  if (coef_f32)
    hipLaunchKernelGGL(assemble_kernel<float2>, dim3(a.nw), dim3(256), 0, st, a, static_cast<float2*>(coef));
  else
    hipLaunchKernelGGL(assemble_kernel<double2>, dim3(a.nw), dim3(256), 0, st, a, static_cast<double2*>(coef));
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// E_mix = sum_w w Re E_L / sum_w w over walkers with w > 0 (fixed order)
__global__ __launch_bounds__(256) void emix_kernel(const double2* __restrict__ eloc, const double* __restrict__ wt,
                                                   int nw, double* __restrict__ out) {
  const int t = threadIdx.x;
  double2 v[1] = {make_double2(0, 0)};
  for (int w = t; w < nw; w += 256) {
    const double ww = wt[w];
    if (ww > 0.0) { v[0].x += ww * eloc[w].x; v[0].y += ww; }
  }
  block_sum<1>(v);
  if (t == 0) out[0] = v[0].y > 0.0 ? v[0].x / v[0].y : 0.0;
}
int launch_emix(const double2* eloc, const double* wt, int nw, double* out, hipStream_t st) {
  hipLaunchKernelGGL(emix_kernel, dim3(1), dim3(256), 0, st, eloc, wt, nw, out);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// Phaseless weight update (one thread per walker):
//   log r = log O' - log O, |I| = |r| exp(Re lfac) exp(dt E_shift),
//   w <- w |I| max(0, cos(Im log r + Im lfac)) (Im lfac: the phase of the
//   background's c-number factor, 0 without one); a walker whose weight is not positive and
//   finite (or whose new overlap is singular) dies and is frozen. The walkers
//   still alive afterwards are exactly those that commit W <- W' (commit_kernel).
__global__ __launch_bounds__(256) void weight_kernel(WeightArgs a, int nw) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  if (w >= nw) return;
  double2 ratio = make_double2(0.0, 0.0);
  if (a.alive[w]) {
    const double2 ln_new = cadd(a.logdet_new[2 * w], a.logdet_new[2 * w + 1]);
    const double2 ln_cur = cadd(a.logdet_cur[2 * w], a.logdet_cur[2 * w + 1]);
    const bool sing = a.sing_new[2 * w] || a.sing_new[2 * w + 1];
    const double2 lr = csub(ln_new, ln_cur);
    const double mag = exp(lr.x);
    ratio = make_double2(mag * cos(lr.y), mag * sin(lr.y));
    const double cs = cos(lr.y + a.lfac[w].y);
    double wn = 0.0;
    if (cs > 0.0) wn = a.weights[w] * exp(lr.x + a.lfac[w].x + a.dt * a.e_shift) * cs;
    if (!sing && wn > 0.0 && isfinite(wn)) {
      if (a.w_cap > 0.0) wn = fmin(wn, a.w_cap);
      a.weights[w] = wn;
    } else {
      a.weights[w] = 0.0;
      a.alive[w] = 0;
      atomicAdd(reinterpret_cast<unsigned long long*>(a.killed), 1ull);
    }
  }
  if (a.ratio_out) a.ratio_out[w] = ratio;
  if (a.weights_out) a.weights_out[w] = a.weights[w];
}

// Walker commit: W <- W' (and the carried S^-1, log det) for every walker
// alive after the weight update; workgroup (x, w) copies elements
// 1024 x .. 1024 x + 1023 of walker w's W' followed by its S^-1 (coalesced,
// 16 bytes per lane and load)
__global__ __launch_bounds__(256) void commit_kernel(WeightArgs a) {
  const int w = blockIdx.y;
  if (!a.alive[w]) return;
  const long per = a.per, sper = a.sinv ? a.sinv_per : 0;
  const long base = (long)blockIdx.x * 1024 + threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long i = base + 256L * u;
    if (i < per) a.W[w * per + i] = a.Wn[w * per + i];
    else if (i - per < sper) a.sinv[w * sper + (i - per)] = a.sinv_new[w * sper + (i - per)];
  }
  if (a.sinv && blockIdx.x == 0 && threadIdx.x < 2) a.logdet_keep[2 * w + threadIdx.x] = a.logdet_new[2 * w + threadIdx.x];
}

// The same commit after the caller exchanged the walker (and S^-1) buffers:
// the new values are already in place for every walker, and the walkers not
// alive after the weight update get their old W (and S^-1, log det) back
__global__ __launch_bounds__(256) void restore_kernel(WeightArgs a) {
  const int w = blockIdx.y;
  if (a.alive[w]) {
    if (a.sinv && blockIdx.x == 0 && threadIdx.x < 2) a.logdet_keep[2 * w + threadIdx.x] = a.logdet_new[2 * w + threadIdx.x];
    return;
  }
  const long per = a.per, sper = a.sinv ? a.sinv_per : 0;
  const long base = (long)blockIdx.x * 1024 + threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long i = base + 256L * u;
    if (i < per) a.W[w * per + i] = a.Wn[w * per + i];
    else if (i - per < sper) a.sinv[w * sper + (i - per)] = a.sinv_new[w * sper + (i - per)];
  }
}

int launch_weights(const WeightArgs& a, int nw, hipStream_t st) {
  hipLaunchKernelGGL(weight_kernel, dim3((nw + 255) / 256), dim3(256), 0, st, a, nw);
  AFQ_TRY_HIP(hipGetLastError());
  const long total = a.per + (a.sinv ? a.sinv_per : 0);
  if (a.swapped) hipLaunchKernelGGL(restore_kernel, dim3((unsigned)((total + 1023) / 1024), nw), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(commit_kernel, dim3((unsigned)((total + 1023) / 1024), nw), dim3(256), 0, st, a);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// Population control by systematic resampling ("comb"). One workgroup: thread 0
// forms the running sums C_i of the weights in walker order (the same
// left-to-right FP64 additions as a sequential cumulative sum) and finds the
// last walker of positive weight; then tooth k at u_k = (k + xi) W / n picks
// the first walker i with C_i > u_k (a tooth at or beyond W picks that last
// walker). out2 = {W, W / n}; W <= 0 leaves src untouched.
__global__ __launch_bounds__(256) void comb_index_kernel(const double* __restrict__ wt, int nw, double xi,
                                                         double* __restrict__ cum, int* __restrict__ src,
                                                         double* __restrict__ out2) {
  __shared__ double total_s;
  __shared__ int last_s;
  const int t = threadIdx.x;
  if (t == 0) {
    double acc = 0.0;
    int last = -1;
    for (int i = 0; i < nw; ++i) {
      acc += wt[i];
      cum[i] = acc;
      if (wt[i] > 0.0) last = i;
    }
    total_s = acc;
    last_s = last;
    out2[0] = acc;
    out2[1] = acc / nw;
  }
  __syncthreads();
  const double total = total_s;
  if (!(total > 0.0) || last_s < 0) return;
  const double step = total / nw;
  for (int k = t; k < nw; k += 256) {
    const double u = ((double)k + xi) * step;
    int lo = 0, hi = nw;                      // first i with cum[i] > u, or nw
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (cum[mid] > u) hi = mid;
      else lo = mid + 1;
    }
    src[k] = lo < last_s ? lo : last_s;
  }
}
int launch_comb_index(const double* weights, int nw, double xi, double* cum, int* src, double* out2,
                      hipStream_t st) {
  hipLaunchKernelGGL(comb_index_kernel, dim3(1), dim3(256), 0, st, weights, nw, xi, cum, src, out2);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// Wout[k] = W[src[k]]; weights[k] = W / n; alive[k] = 1
__global__ __launch_bounds__(256) void comb_apply_kernel(const double2* __restrict__ W, double2* __restrict__ Wout,
                                                         long per, const int* __restrict__ src,
                                                         const double* __restrict__ out2, double* weights,
                                                         int* alive) {
  const int k = blockIdx.y;
  const double2* from = W + (long)src[k] * per;
  double2* to = Wout + (long)k * per;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < per; i += (long)gridDim.x * 256) to[i] = from[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    weights[k] = out2[1];
    alive[k] = 1;
  }
}
int launch_comb_apply(const double2* W, double2* Wout, long per, int nw, const int* src, const double* out2,
                      double* weights, int* alive, hipStream_t st) {
  const int bx = (int)std::min<long>(ceil_div(per, 256), 64);
  hipLaunchKernelGGL(comb_apply_kernel, dim3(bx, nw), dim3(256), 0, st, W, Wout, per, src, out2, weights, alive);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// max |x_ij - x_ji| and max |x_ij| over a batch of square matrices, and
// max |Im z| of a complex array (input validation at system creation)
__global__ void asym_kernel(const double* __restrict__ x, int M, long nmat, double* out) {
  __shared__ double red[2][256];
  double a = 0.0, m = 0.0;
  const long total = nmat * M * M;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long b = i / ((long)M * M);
    const int r = (int)((i / M) % M), c = (int)(i % M);
    const double v = x[i];
    const double vt = x[b * M * M + (long)c * M + r];
    a = fmax(a, fabs(v - vt));
    m = fmax(m, fabs(v));
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // non-negative doubles order like their bit patterns
    atomicMax(reinterpret_cast<unsigned long long*>(out), __double_as_longlong(red[0][0]));
    atomicMax(reinterpret_cast<unsigned long long*>(out + 1), __double_as_longlong(red[1][0]));
  }
}
__global__ void imag_kernel(const double2* __restrict__ z, long n, double* out) {
  __shared__ double red[256];
  double a = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a = fmax(a, fabs(z[i].y));
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(reinterpret_cast<unsigned long long*>(out), __double_as_longlong(red[0]));
}
int launch_asym(const double* x, int M, long nmat, double* out2, hipStream_t st) {
  hipLaunchKernelGGL(asym_kernel, dim3(grid_for(nmat * M * M) > 1024 ? 1024 : grid_for(nmat * M * M)), dim3(256), 0,
                     st, x, M, nmat, out2);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
int launch_maximag(const double2* z, long n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(imag_kernel, dim3(grid_for(n) > 1024 ? 1024 : grid_for(n)), dim3(256), 0, st, z, n, out);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// infinity norm (max absolute row sum) of a real M x M matrix
__global__ void infnorm_kernel(const double* __restrict__ x, int M, double* out) {
  __shared__ double red[256];
  double a = 0.0;
  for (int r = threadIdx.x; r < M; r += 256) {
    double s = 0.0;
    for (int c = 0; c < M; ++c) s += fabs(x[(long)r * M + c]);
    a = fmax(a, s);
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}
int launch_infnorm(const double* x, int M, double* out, hipStream_t st) {
  hipLaunchKernelGGL(infnorm_kernel, dim3(1), dim3(256), 0, st, x, M, out);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// log overlap per walker = sum of the two spin log-determinants
__global__ void logovlp_kernel(const double2* __restrict__ ld, int nw, double2* __restrict__ out) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nw) out[w] = cadd(ld[2 * w], ld[2 * w + 1]);
}
int launch_logovlp(const double2* ld, int nw, double2* out, hipStream_t st) {
  hipLaunchKernelGGL(logovlp_kernel, dim3(ceil_div(nw, 256)), dim3(256), 0, st, ld, nw, out);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// flags: alive[w] = weight[w] > 0 && !singular
__global__ void init_alive_kernel(const double* __restrict__ wt, const int* __restrict__ sing, int nw,
                                  int* __restrict__ alive, int* __restrict__ bad) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const int a = wt[w] > 0.0;
  alive[w] = a;
  if (a && (sing[2 * w] || sing[2 * w + 1])) atomicAdd(bad, 1);
}
int launch_init_alive(const double* wt, const int* sing, int nw, int* alive, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(init_alive_kernel, dim3(ceil_div(nw, 256)), dim3(256), 0, st, wt, sing, nw, alive, bad);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// step counter kept on the device, so captured launch sequences advance it
__global__ void counter_kernel(uint64_t* c, uint64_t v, int add) {
  if (threadIdx.x == 0) *c = add ? *c + v : v;
}
int counter_add(uint64_t* c, uint64_t v, hipStream_t st) {
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, st, c, v, 1);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
int counter_set(uint64_t* c, uint64_t v, hipStream_t st) {
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, st, c, v, 0);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// ---------------------------------------------------------------------------
// back-propagation window
// ---------------------------------------------------------------------------
// dst = conj(src), n complex elements (the coefficients of B^H = B1 T_K(A^H) B1)
template <typename C>
__global__ void conj_copy_kernel(const C* __restrict__ src, C* __restrict__ dst, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    C v = src[i];
    v.y = -v.y;
    dst[i] = v;
  }
}
int launch_conj_copy(const void* src, void* dst, long n, bool f32, hipStream_t st) {
  if (n <= 0) return AFQ_OK;
  if (f32)
    hipLaunchKernelGGL(conj_copy_kernel<float2>, dim3(grid_for(n)), dim3(256), 0, st,
                       static_cast<const float2*>(src), static_cast<float2*>(dst), n);
  else
    hipLaunchKernelGGL(conj_copy_kernel<double2>, dim3(grid_for(n)), dim3(256), 0, st,
                       static_cast<const double2*>(src), static_cast<double2*>(dst), n);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// dst[slab][k] = src[slab][idx[k]] for rows of rw 8-byte words, nrows rows a slab
__global__ void gather_rows_kernel(const uint2* __restrict__ src, uint2* __restrict__ dst, long rw, int nrows,
                                   const int* __restrict__ idx, long total) {
  for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    const long row = t / rw, e = t - row * rw;
    const long slab = row / nrows;
    const int k = (int)(row - slab * nrows);
    dst[t] = src[(slab * nrows + idx[k]) * rw + e];
  }
}
int launch_gather_rows(const void* src, void* dst, long row_bytes, int nrows, int nslabs, const int* idx,
                       hipStream_t st) {
  AFQ_CHECK(row_bytes % 8 == 0, AFQ_E_INVALID, "gather_rows: row size is not a multiple of 8 bytes");
  const long rw = row_bytes / 8, total = rw * nrows * (long)nslabs;
  if (total == 0) return AFQ_OK;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for(total)), dim3(256), 0, st, static_cast<const uint2*>(src),
                     static_cast<uint2*>(dst), rw, nrows, idx, total);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// stats[0] = sum of the positive weights (fixed order), stats[1] = number of
// walkers of positive weight whose bra-ket overlap is singular in either spin
__global__ __launch_bounds__(256) void bp_stats_kernel(const double* __restrict__ wt, const int* __restrict__ sing,
                                                       int nw, double* __restrict__ stats) {
  const int t = threadIdx.x;
  double2 v[1] = {make_double2(0, 0)};
  for (int w = t; w < nw; w += 256) {
    const double ww = wt[w];
    if (ww > 0.0) {
      v[0].x += ww;
      v[0].y += (sing[2 * w] || sing[2 * w + 1]) ? 1.0 : 0.0;
    }
  }
  block_sum<1>(v);
  if (t == 0) { stats[0] = v[0].x; stats[1] = v[0].y; }
}
int launch_bp_stats(const double* wt, const int* sing, int nw, double* stats, hipStream_t st) {
  hipLaunchKernelGGL(bp_stats_kernel, dim3(1), dim3(256), 0, st, wt, sing, nw, stats);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

// Operands of P^s = Q Y^T over the walker-stacked index r = w n + a:
//   Y[i][r] <- f_w Y[i][r],  Q[i][r] = conj(psi_w[i][off + a])   (f_w = w_w / sum w)
// and both zero for walkers of weight <= 0 (whatever their Y or psi hold).
__global__ void bp_pack_kernel(double2* __restrict__ Y, double2* __restrict__ Q, const double2* __restrict__ psi,
                               long per, int ntot, int off, int n, int nw, const double* __restrict__ wt,
                               const double* __restrict__ stats, long total) {
  const long K = (long)nw * n;
  const double inv = stats[0] > 0.0 ? 1.0 / stats[0] : 0.0;
  for (long t = blockIdx.x * 256L + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    const long i = t / K, r = t - i * K;
    const int w = (int)(r / n), a = (int)(r - (long)w * n);
    const double ww = wt[w];
    if (ww > 0.0) {
      Y[t] = cscale(Y[t], ww * inv);
      Q[t] = cconj(psi[w * per + i * ntot + off + a]);
    } else {
      Y[t] = make_double2(0.0, 0.0);
      Q[t] = make_double2(0.0, 0.0);
    }
  }
}
int launch_bp_pack(double2* Y, double2* Q, const double2* psi, long per, int ntot, int off, int n, int nw, int M,
                   const double* wt, const double* stats, hipStream_t st) {
  const long total = (long)M * nw * n;
  if (total == 0) return AFQ_OK;
  hipLaunchKernelGGL(bp_pack_kernel, dim3(grid_for(total)), dim3(256), 0, st, Y, Q, psi, per, ntot, off, n, nw, wt,
                     stats, total);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
