// Orthogonal multi-determinant trial (multi-determinant paragraph of the AFQMC
// section): psi_T = sum_I c_I |D_I>, every D_I the reference determinant
// (the first n columns of an orthonormal basis C, per spin) with k <= 4 hole
// orbitals replaced slot by slot by particle orbitals.
//
// Everything is expressed through the reference: with Theta = W S0^-1,
// T = C^H Theta is the identity on the reference rows, and the ratio
// <D_I|W>/<D_0|W> of one spin is det A with A[q][r] = T[p_q][h_r] (k x k,
// the Sherman-Morrison-Woodbury form of the rank-k change of the overlap).
// For a one-body operator L, with R_I the rows O_I of [T^H; C_V^H] L Theta,
//   det(M_I + e R_I) = det(I + e Omega0) det(A + e Y1 + e^2 Y2) + O(e^3)
// where Omega0 = T^H L Theta (reference block), and over the active virtual
// rows V and hole columns h
//   Y1 = (Omega_V - T_V Omega0)[p, h],   Y2 = -((Omega_V - T_V Omega0) Omega0)[p, h].
// Its e^1 coefficient is R_I tr Omega_I (the ratio-weighted trace of the
// determinant's half-rotated Omega) and twice its e^2 coefficient is
// R_I [(tr Omega_I)^2 - tr Omega_I^2]; both are polynomials in A, Y1, Y2
// (first- and second-order cofactor expansions), so no determinant's A is
// ever inverted and a walker orthogonal to some D_I is handled exactly. The
// mixed energy and force bias are then ratio-weighted sums over determinants:
//   <psi|W> = <D_0|W> sum_I conj(c_I) R_I,
//   E_L = e_core + sum_I conj(c_I) [N1^h + sum_g N2^g] / sum_I conj(c_I) R_I,
//   vbar_g = sum_I conj(c_I) N1^g / sum_I conj(c_I) R_I,
// with, per determinant and operator (spins u, d):
//   N1 = N1_u R_d + R_u N1_d,   N2 = (P2_u R_d + R_u P2_d + 2 N1_u N1_d) / 2.
// The determinant of A + e Y1 + e^2 Y2 is taken in truncated polynomial
// arithmetic (three coefficients per entry, Laplace expansion for k <= 4), which
// yields det A, its first- and second-order changes at once.
// Work per step: one FP64 MFMA GEMM per walker chunk over (X + 1) operators
// (L^g and h1) and the reference plus active-virtual rows (shared by both
// spins), then one workgroup per (walker, operator) that stages its blocks in
// LDS for the small products, the per-excitation polynomials and the
// determinant sums.
#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <vector>
#include "common.h"
#include "step_kernels.h"
#include "trace.h"

constexpr int MSD_MAX_N = 64;       // electrons per spin
constexpr int MSD_MAX_NO = 16;      // active holes per spin
constexpr int MSD_MAX_NV = 32;      // active virtual orbitals
constexpr int MSD_MAX_EXC = 256;    // distinct excitations per spin
constexpr size_t MSD_MAX_LDS = 160 * 1024;
constexpr size_t MSD_OMEGA_BUDGET = size_t(4) << 30;   // bytes of Omega per walker chunk

// ---------------------------------------------------------------------------
// truncated polynomials a + b e + c e^2 and their k x k determinants (k <= 4)
// ---------------------------------------------------------------------------
struct P3 {
  double2 a, b, c;
};
__device__ inline P3 pmul(const P3& x, const P3& y) {
  return {cmul(x.a, y.a), cadd(cmul(x.a, y.b), cmul(x.b, y.a)),
          cadd(cadd(cmul(x.a, y.c), cmul(x.b, y.b)), cmul(x.c, y.a))};
}
__device__ inline P3 padd(const P3& x, const P3& y) { return {cadd(x.a, y.a), cadd(x.b, y.b), cadd(x.c, y.c)}; }
__device__ inline P3 psub(const P3& x, const P3& y) { return {csub(x.a, y.a), csub(x.b, y.b), csub(x.c, y.c)}; }
__device__ inline P3 pdet2(const P3& a, const P3& b, const P3& c, const P3& d) { return psub(pmul(a, d), pmul(b, c)); }

__device__ P3 pdet(const P3 (&m)[MSD_KMAX][MSD_KMAX], int k) {
  const double2 z = make_double2(0.0, 0.0);
  if (k == 0) return {make_double2(1.0, 0.0), z, z};
  if (k == 1) return m[0][0];
  if (k == 2) return pdet2(m[0][0], m[0][1], m[1][0], m[1][1]);
  if (k == 3) {
    const P3 c0 = pdet2(m[1][1], m[1][2], m[2][1], m[2][2]);
    const P3 c1 = pdet2(m[1][0], m[1][2], m[2][0], m[2][2]);
    const P3 c2 = pdet2(m[1][0], m[1][1], m[2][0], m[2][1]);
    return padd(psub(pmul(m[0][0], c0), pmul(m[0][1], c1)), pmul(m[0][2], c2));
  }
  // k = 4: Laplace expansion along rows (0, 1) with the complementary minors of rows (2, 3)
  P3 acc = {z, z, z};
  const int cp[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (int t = 0; t < 6; ++t) {
    const int a = cp[t][0], b = cp[t][1], c = cp[5 - t][0], d = cp[5 - t][1];
    const P3 top = pdet2(m[0][a], m[0][b], m[1][a], m[1][b]);
    const P3 bot = pdet2(m[2][c], m[2][d], m[3][c], m[3][d]);
    const P3 term = pmul(top, bot);
    // sign (-1)^(0 + 1 + a + b): pairs (0,2) and (1,3) are negative
    acc = (t == 1 || t == 4) ? psub(acc, term) : padd(acc, term);
  }
  return acc;
}

// det(A + e Y1 + e^2 Y2) for one excitation of rank K, entries read from LDS:
// A[q][r] = T[v_q][col_r], Y[q][r] = Y[v_q][hs_r] (v: particle slots, col:
// hole columns, hs: hole slots)
template <int K>
__device__ P3 pdet_lds(const double2* T, const double2* Y1, const double2* Y2, int n, int no, const int* ex) {
  int v[K > 0 ? K : 1], col[K > 0 ? K : 1], hs[K > 0 ? K : 1];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    v[q] = ex[1 + MSD_KMAX + q];
    col[q] = ex[1 + 2 * MSD_KMAX + q];
    hs[q] = ex[1 + q];
  }
  auto E = [&](int q, int r) -> P3 {
    const int yi = v[q] * no + hs[r];
    return {T[v[q] * n + col[r]], Y1[yi], Y2[yi]};
  };
  const double2 z = make_double2(0.0, 0.0);
  if constexpr (K == 0) {
    return {make_double2(1.0, 0.0), z, z};
  } else if constexpr (K == 1) {
    return E(0, 0);
  } else if constexpr (K == 2) {
    return pdet2(E(0, 0), E(0, 1), E(1, 0), E(1, 1));
  } else if constexpr (K == 3) {
    const P3 c0 = pdet2(E(1, 1), E(1, 2), E(2, 1), E(2, 2));
    const P3 c1 = pdet2(E(1, 0), E(1, 2), E(2, 0), E(2, 2));
    const P3 c2 = pdet2(E(1, 0), E(1, 1), E(2, 0), E(2, 1));
    return padd(psub(pmul(E(0, 0), c0), pmul(E(0, 1), c1)), pmul(E(0, 2), c2));
  } else {
    // expansion along row 0 into 3 x 3 minors of rows 1..3, one at a time
    // (keeps the register footprint of the rank-3 path)
    P3 acc = {z, z, z};
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
      const int c0 = j == 0 ? 1 : 0, c1 = j <= 1 ? 2 : 1, c2 = j <= 2 ? 3 : 2;
      const P3 m0 = pdet2(E(2, c1), E(2, c2), E(3, c1), E(3, c2));
      const P3 m1 = pdet2(E(2, c0), E(2, c2), E(3, c0), E(3, c2));
      const P3 m2 = pdet2(E(2, c0), E(2, c1), E(3, c0), E(3, c1));
      const P3 minor = padd(psub(pmul(E(1, c0), m0), pmul(E(1, c1), m1)), pmul(E(1, c2), m2));
      const P3 term = pmul(E(0, j), minor);
      acc = (j & 1) ? psub(acc, term) : padd(acc, term);
    }
    return acc;
  }
}

// fixed-order sum of one complex value over a 256-thread workgroup (wave
// butterflies, then the four wave sums in order); every thread gets the total
__device__ inline double2 wg_sum(double2 v, double2* scratch4) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  const int t = threadIdx.x;
  if ((t & 63) == 0) scratch4[t >> 6] = v;
  __syncthreads();
  const double2 r = cadd(cadd(scratch4[0], scratch4[1]), cadd(scratch4[2], scratch4[3]));
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// per (walker, excitation): det A, A[q][r] = T_V[p_q][h_r]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void msd_ratio_kernel(const double2* __restrict__ tv, int nv, int ntot, int off,
                                                       const int* __restrict__ exc, int nexc,
                                                       double2* __restrict__ d0) {
  const int e = blockIdx.x * 64 + threadIdx.x, w = blockIdx.y;
  if (e >= nexc) return;
  const int* ex = exc + e * MSD_EXC;
  const int k = ex[0];
  const double2* T = tv + (long)w * nv * ntot + off;
  const double2 z = make_double2(0.0, 0.0);
  P3 m[MSD_KMAX][MSD_KMAX];
  for (int q = 0; q < MSD_KMAX; ++q)
    for (int r = 0; r < MSD_KMAX; ++r)
      m[q][r] = {(q < k && r < k) ? T[(long)ex[1 + MSD_KMAX + q] * ntot + ex[1 + 2 * MSD_KMAX + r]] : z, z, z};
  d0[(long)w * nexc + e] = pdet(m, k).a;
}

// ---------------------------------------------------------------------------
// per walker: den = sum_I conj(c_I) R_I(up) R_I(down); logdet[2w] += log den
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_den_kernel(const double2* __restrict__ cconj, const int* __restrict__ pair,
                                                      int ndet, const double2* __restrict__ d0u, int nexc0,
                                                      const double2* __restrict__ d0d, int nexc1,
                                                      double2* __restrict__ den, double2* __restrict__ logdet) {
  const int w = blockIdx.x, t = threadIdx.x;
  __shared__ double2 red[256];
  double2 acc = make_double2(0.0, 0.0);
  for (int I = t; I < ndet; I += 256) {
    const double2 ru = d0u[(long)w * nexc0 + pair[2 * I]];
    const double2 rd = d0d[(long)w * nexc1 + pair[2 * I + 1]];
    acc = cadd(acc, cmul(cconj[I], cmul(ru, rd)));
  }
  red[t] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = cadd(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) {
    den[w] = red[0];
    logdet[2 * w] = cadd(logdet[2 * w], clog(red[0]));
  }
}

// ---------------------------------------------------------------------------
// per (walker, excitation of one spin): the operator-independent coefficient
// of that excitation in the determinant sums,
//   S_u[e] = sum_{I: up(I) = e} conj(c_I) R_d(I),  S_d[e] = sum_{I: dn(I) = e} conj(c_I) R_u(I)
// (determinants grouped per excitation on the host, summed in index order)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_pairsum_kernel(const double2* __restrict__ cconj,
                                                          const int* __restrict__ pair,
                                                          const int* __restrict__ off0, const int* __restrict__ det0,
                                                          const int* __restrict__ off1, const int* __restrict__ det1,
                                                          const double2* __restrict__ d0u, int nexc0,
                                                          const double2* __restrict__ d0d, int nexc1,
                                                          double2* __restrict__ su, double2* __restrict__ sd) {
  const int w = blockIdx.x, t = threadIdx.x;
  for (int e = t; e < nexc0 + nexc1; e += 256) {
    const bool up = e < nexc0;
    const int x = up ? e : e - nexc0;
    const int* off = up ? off0 : off1;
    const int* det = up ? det0 : det1;
    const double2* other = up ? d0d + (long)w * nexc1 : d0u + (long)w * nexc0;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = off[x]; j < off[x + 1]; ++j) {
      const int I = det[j];
      acc = cadd(acc, cmul(cconj[I], other[pair[2 * I + (up ? 1 : 0)]]));
    }
    if (up) su[(long)w * nexc0 + x] = acc;
    else sd[(long)w * nexc1 + x] = acc;
  }
}

// ---------------------------------------------------------------------------
// one workgroup per (walker of the chunk, operator g in [0, X]): both spins'
// small products, per-excitation polynomials, then the determinant sums
// ---------------------------------------------------------------------------
struct MsdPostArgs {
  const double2* omega;      // (X + 1) nr rows x ldo columns (walker-major, ntot per walker)
  long ldo;
  const double2* tv;         // nw x nv x ntot
  const int* exc[2];
  const int* hact[2];
  int n[2], off[2], no[2], nexc[2];
  int nmax, nv, nr, ntot, nexc_max;
  const double2* S[2];       // nw x nexc: operator-independent coefficients per excitation
  const int* pair;
  const double2* cconj;
  int ndet, X, w0;
  double2* num;              // nw x (2X + 1)
};

__global__ __launch_bounds__(256) void msd_post_kernel(MsdPostArgs a) {
  extern __shared__ double2 lds[];
  const int g = blockIdx.x, wl = blockIdx.y, w = a.w0 + wl, t = threadIdx.x;
  const int nv = a.nv;
  // persistent: N1 per spin and excitation (for the cross-spin term); reduction scratch
  double2* N1 = lds;
  double2* red = N1 + 2 * a.nexc_max;          // 4 wave partials (x 2)
  double2* work = red + 8;
  // linear terms: sum_e N1[e] S[e] (force bias) and sum_e P2[e] S[e] / 2 (two-body)
  double2 av = make_double2(0.0, 0.0), ae = make_double2(0.0, 0.0);
  for (int sp = 0; sp < 2; ++sp) {
    const int n = a.n[sp], no = a.no[sp], off = a.off[sp];
    double2* Om = work;                         // (n + nv) x n: reference rows, then virtual rows
    double2* T = Om + (n + nv) * n;             // nv x n
    double2* P = T + nv * n;                    // n x no: Omega0[:, h]
    double2* Q = P + n * no;                    // n x no: Omega0 P
    double2* Y1 = Q + n * no;                   // nv x no
    double2* Y2 = Y1 + nv * no;                 // nv x no
    const double2* src = a.omega + (long)g * a.nr * a.ldo + (long)wl * a.ntot + off;
    for (int e = t; e < (n + nv) * n; e += 256) {
      const int r = e / n, j = e - r * n;
      const int ru = r < n ? r : a.nmax + (r - n);
      Om[e] = src[(long)ru * a.ldo + j];
    }
    const double2* tvw = a.tv + (long)w * nv * a.ntot + off;
    for (int e = t; e < nv * n; e += 256) {
      const int v = e / n, j = e - v * n;
      T[e] = tvw[(long)v * a.ntot + j];
    }
    __syncthreads();
    // traces of the reference block: t0 = tr Omega0, q0 = tr Omega0^2; P = Omega0[:, h]
    double2 t0 = make_double2(0.0, 0.0), q0 = make_double2(0.0, 0.0);
    for (int i = t; i < n; i += 256) t0 = cadd(t0, Om[i * n + i]);
    for (int e = t; e < n * n; e += 256) {
      const int i = e / n, j = e - i * n;
      q0 = cadd(q0, cmul(Om[i * n + j], Om[j * n + i]));
    }
    const int* hact = a.hact[sp];
    for (int e = t; e < n * no; e += 256) {
      const int l = e / no, hh = e - l * no;
      P[e] = Om[l * n + hact[hh]];
    }
    t0 = wg_sum(t0, red);
    q0 = wg_sum(q0, red + 4);
    // Q = Omega0 P
    for (int e = t; e < n * no; e += 256) {
      const int l = e / no, hh = e - l * no;
      double2 acc = make_double2(0.0, 0.0);
      for (int j = 0; j < n; ++j) acc = cadd(acc, cmul(Om[l * n + j], P[j * no + hh]));
      Q[e] = acc;
    }
    __syncthreads();
    // Y1 = Omega_V[:, h] - T_V P ;  Y2 = T_V Q - Omega_V P
    for (int e = t; e < nv * no; e += 256) {
      const int v = e / no, hh = e - v * no;
      const double2* ov = Om + (n + v) * n;
      const double2* tv = T + v * n;
      double2 y1 = ov[hact[hh]], y2 = make_double2(0.0, 0.0);
      for (int l = 0; l < n; ++l) {
        const double2 p = P[l * no + hh];
        y1 = csub(y1, cmul(tv[l], p));
        y2 = cadd(y2, csub(cmul(tv[l], Q[l * no + hh]), cmul(ov[l], p)));
      }
      Y1[e] = y1;
      Y2[e] = y2;
    }
    __syncthreads();
    // per excitation: det(A + e Y1 + e^2 Y2) = d0 + d1 e + d2 e^2 (excitations
    // are sorted by rank, so a wave mostly runs one of the five paths)
    const double2* Sw = a.S[sp] + (long)w * a.nexc[sp];
    for (int e = t; e < a.nexc[sp]; e += 256) {
      const int* ex = a.exc[sp] + e * MSD_EXC;
      P3 d;
      switch (ex[0]) {
        case 0: d = pdet_lds<0>(T, Y1, Y2, n, no, ex); break;
        case 1: d = pdet_lds<1>(T, Y1, Y2, n, no, ex); break;
        case 2: d = pdet_lds<2>(T, Y1, Y2, n, no, ex); break;
        case 3: d = pdet_lds<3>(T, Y1, Y2, n, no, ex); break;
        default: d = pdet_lds<4>(T, Y1, Y2, n, no, ex); break;
      }
      const double2 n1 = cadd(d.b, cmul(t0, d.a));
      // P2 / 2 = d2 + t0 d1 + (t0^2 - q0) d0 / 2
      const double2 p2h = cadd(cadd(d.c, cmul(t0, d.b)), cscale(cmul(csub(cmul(t0, t0), q0), d.a), 0.5));
      N1[sp * a.nexc_max + e] = n1;
      const double2 se = Sw[e];
      av = cadd(av, cmul(n1, se));
      ae = cadd(ae, cmul(p2h, se));
    }
    __syncthreads();
  }
  // cross-spin term of the two-body sum: sum_I conj(c_I) N1_u N1_d
  for (int I = t; I < a.ndet; I += 256) {
    const double2 n1u = N1[a.pair[2 * I]], n1d = N1[a.nexc_max + a.pair[2 * I + 1]];
    ae = cadd(ae, cmul(a.cconj[I], cmul(n1u, n1d)));
  }
  av = wg_sum(av, red);
  ae = wg_sum(ae, red + 4);
  if (t == 0) {
    double2* out = a.num + (long)w * (2 * a.X + 1);
    if (g < a.X) {
      out[g] = av;
      out[a.X + g] = ae;
    } else {
      out[2 * a.X] = av;
    }
  }
}

// per walker: parts = (E1, E2, 0) and vbar from the numerators and den
__global__ __launch_bounds__(256) void msd_finish_kernel(const double2* __restrict__ num,
                                                         const double2* __restrict__ den, int X,
                                                         double2* __restrict__ parts, double2* __restrict__ vbar) {
  const int w = blockIdx.x, t = threadIdx.x;
  __shared__ double2 red[256];
  const double2* nw_ = num + (long)w * (2 * X + 1);
  const double2 d = den[w];
  double2 acc = make_double2(0.0, 0.0);
  for (int g = t; g < X; g += 256) {
    vbar[(long)w * X + g] = cdiv(nw_[g], d);
    acc = cadd(acc, nw_[X + g]);
  }
  red[t] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = cadd(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) {
    parts[3 * w] = cdiv(nw_[2 * X], d);
    parts[3 * w + 1] = cdiv(red[0], d);
    parts[3 * w + 2] = make_double2(0.0, 0.0);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static size_t msd_lds_bytes(afq_system s) {
  size_t spin = 0;
  const size_t nv = s->msd_nv;
  for (int sp = 0; sp < 2; ++sp) {
    const size_t n = s->nspin_n(sp), no = s->msd_no[sp];
    spin = std::max(spin, (n + nv) * n + nv * n + 2 * n * no + 2 * nv * no);
  }
  const size_t nexc = std::max(s->msd_nexc[0], s->msd_nexc[1]);
  return (2 * nexc + 8 + spin) * 16;
}

int msd_set(afq_system s, const double* C, int n_det, const double* coeffs, const int32_t* exc) {
  hipStream_t st = s->stream;
  const int M = s->M, X = s->X;
  if (n_det == 0) {
    if (s->msd_n) ++s->version;
    s->msd_n = 0;
    return eri_sync(s);
  }
  AFQ_CHECK(n_det >= 1 && n_det <= 65536, AFQ_E_INVALID, "afq_system_set_msd: n_det must be in [0, 65536]");
  AFQ_CHECK(C && coeffs && exc, AFQ_E_INVALID, "afq_system_set_msd: NULL input");
  AFQ_CHECK(s->prec == AFQ_FP64, AFQ_E_UNSUPPORTED, "afq_system_set_msd: multi-determinant trials run in FP64 mode");
  AFQ_CHECK(s->n_up <= MSD_MAX_N && s->n_dn <= MSD_MAX_N, AFQ_E_UNSUPPORTED,
            "afq_system_set_msd: at most 64 electrons per spin");
  // the basis must be orthonormal and its first columns must be the trial's spin blocks
  std::vector<double2> hC((size_t)M * M), hphi((size_t)M * s->ntot);
  AFQ_TRY_HIP(hipMemcpyAsync(hC.data(), C, hC.size() * 16, hipMemcpyDeviceToHost, st));
  AFQ_TRY_HIP(hipMemcpyAsync(hphi.data(), s->phi.p, hphi.size() * 16, hipMemcpyDeviceToHost, st));
  AFQ_TRY_HIP(hipStreamSynchronize(st));
  for (int sp = 0; sp < 2; ++sp) {
    const int n = s->nspin_n(sp), off = s->spin_off(sp);
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < n; ++j) {
        const double2 a = hC[(size_t)i * M + j], b = hphi[(size_t)i * s->ntot + off + j];
        AFQ_CHECK(std::fabs(a.x - b.x) <= 1e-12 && std::fabs(a.y - b.y) <= 1e-12, AFQ_E_INVALID,
                  "afq_system_set_msd: the first n columns of C must equal the trial's spin block");
      }
  }
  {
    DevBuf gram;
    AFQ_RET(gram.alloc((size_t)M * M * 16));
    GemmArgs<double> g = gemm_args<double>();
    g.m = M; g.n = M; g.k = M;
    g.A = C; g.lda = M; g.opA = OP_C; g.cA = true;
    g.B = C; g.ldb = M; g.cB = true;
    g.C = gram.as<double>(); g.ldc = M; g.cC = true;
    AFQ_RET(gemm<double>(g, st));
    std::vector<double2> hg((size_t)M * M);
    AFQ_TRY_HIP(hipMemcpyAsync(hg.data(), gram.p, hg.size() * 16, hipMemcpyDeviceToHost, st));
    AFQ_TRY_HIP(hipStreamSynchronize(st));
    double dev = 0.0;
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        const double2 v = hg[(size_t)i * M + j];
        dev = std::max(dev, std::hypot(v.x - (i == j ? 1.0 : 0.0), v.y));
      }
    AFQ_CHECK(dev <= 1e-10, AFQ_E_INVALID, "afq_system_set_msd: C is not orthonormal (|C^H C - I| > 1e-10)");
  }
  // excitations: validate; collect active holes per spin, active virtuals (both
  // spins) and the distinct excitations of each spin
  std::set<std::vector<int>> seen;
  std::vector<int> hpair((size_t)2 * n_det);
  std::vector<std::vector<int>> hact(2);
  std::vector<int> vact;
  std::vector<std::map<std::vector<int>, int>> uniq(2);
  std::vector<std::vector<std::vector<int>>> ulist(2);
  for (int I = 0; I < n_det; ++I) {
    std::vector<int> occ;
    for (int sp = 0; sp < 2; ++sp) {
      const int32_t* r = exc + ((size_t)I * 2 + sp) * 9;
      const int k = r[0], n = s->nspin_n(sp);
      AFQ_CHECK(k >= 0 && k <= MSD_KMAX && k <= n, AFQ_E_UNSUPPORTED,
                "afq_system_set_msd: excitation rank must be in [0, 4] and at most the electron count");
      std::vector<int> e(1 + 2 * k);
      e[0] = k;
      std::set<int> hs, ps;
      for (int q = 0; q < k; ++q) {
        const int h = r[1 + q], p = r[1 + MSD_KMAX + q];
        AFQ_CHECK(h >= 0 && h < n && p >= n && p < M, AFQ_E_INVALID,
                  "afq_system_set_msd: holes must be reference orbitals and particles virtual orbitals");
        AFQ_CHECK(hs.insert(h).second && ps.insert(p).second, AFQ_E_INVALID,
                  "afq_system_set_msd: repeated hole or particle in one excitation");
        e[1 + q] = h;
        e[1 + k + q] = p;
        if (std::find(hact[sp].begin(), hact[sp].end(), h) == hact[sp].end()) hact[sp].push_back(h);
        if (std::find(vact.begin(), vact.end(), p) == vact.end()) vact.push_back(p);
      }
      auto it = uniq[sp].find(e);
      if (it == uniq[sp].end()) {
        it = uniq[sp].emplace(e, (int)ulist[sp].size()).first;
        ulist[sp].push_back(e);
      }
      hpair[2 * I + sp] = it->second;
      // the occupation set decides orthogonality; the slot pairing only fixes the sign
      occ.push_back(-1 - sp);
      occ.insert(occ.end(), hs.begin(), hs.end());
      occ.push_back(-10 - sp);
      occ.insert(occ.end(), ps.begin(), ps.end());
    }
    AFQ_CHECK(seen.insert(occ).second, AFQ_E_INVALID,
              "afq_system_set_msd: two determinants have the same occupation (the expansion must be orthogonal)");
  }
  // order each spin's excitations by rank (waves of the sums kernel then take one rank path)
  for (int sp = 0; sp < 2; ++sp) {
    std::vector<int> order(ulist[sp].size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ulist[sp][x][0] < ulist[sp][y][0]; });
    std::vector<int> where(order.size());
    std::vector<std::vector<int>> sorted(order.size());
    for (size_t i = 0; i < order.size(); ++i) {
      where[order[i]] = (int)i;
      sorted[i] = ulist[sp][order[i]];
    }
    ulist[sp].swap(sorted);
    for (int I = 0; I < n_det; ++I) hpair[2 * I + sp] = where[hpair[2 * I + sp]];
  }
  for (int sp = 0; sp < 2; ++sp) {
    AFQ_CHECK((int)hact[sp].size() <= MSD_MAX_NO && (int)ulist[sp].size() <= MSD_MAX_EXC, AFQ_E_UNSUPPORTED,
              "afq_system_set_msd: at most 16 active holes and 256 distinct excitations per spin");
    std::sort(hact[sp].begin(), hact[sp].end());
  }
  AFQ_CHECK((int)vact.size() <= MSD_MAX_NV, AFQ_E_UNSUPPORTED, "afq_system_set_msd: at most 32 active virtuals");
  std::sort(vact.begin(), vact.end());
  const int nv = (int)vact.size(), nmax = std::max(s->n_up, s->n_dn), nr = nmax + nv;
  // tentative sizes for the LDS check
  const int old_no[2] = {s->msd_no[0], s->msd_no[1]}, old_nexc[2] = {s->msd_nexc[0], s->msd_nexc[1]};
  const int old_nv = s->msd_nv;
  for (int sp = 0; sp < 2; ++sp) {
    s->msd_no[sp] = (int)hact[sp].size();
    s->msd_nexc[sp] = (int)ulist[sp].size();
  }
  s->msd_nv = nv;
  const size_t lds = msd_lds_bytes(s);
  if (lds > MSD_MAX_LDS) {
    for (int sp = 0; sp < 2; ++sp) { s->msd_no[sp] = old_no[sp]; s->msd_nexc[sp] = old_nexc[sp]; }
    s->msd_nv = old_nv;
    afq_set_error("afq_system_set_msd: the expansion needs more than 160 KB of LDS per workgroup");
    return AFQ_E_UNSUPPORTED;
  }
  s->msd_n = 0;   // detached until the tables below are complete
  // device tables
  std::vector<double2> cc(n_det);
  for (int I = 0; I < n_det; ++I) {
    cc[I] = make_double2(coeffs[2 * I], -coeffs[2 * I + 1]);
    AFQ_CHECK(std::isfinite(cc[I].x) && std::isfinite(cc[I].y), AFQ_E_INVALID,
              "afq_system_set_msd: a coefficient is not finite");
  }
  AFQ_RET(s->msd_cconj.alloc((size_t)n_det * 16));
  AFQ_RET(s->msd_pair.alloc((size_t)n_det * 2 * sizeof(int)));
  AFQ_TRY_HIP(hipMemcpyAsync(s->msd_cconj.p, cc.data(), cc.size() * 16, hipMemcpyHostToDevice, st));
  AFQ_TRY_HIP(hipMemcpyAsync(s->msd_pair.p, hpair.data(), hpair.size() * sizeof(int), hipMemcpyHostToDevice, st));
  std::vector<std::vector<int>> dexc(2);
  for (int sp = 0; sp < 2; ++sp) {
    const int no = (int)hact[sp].size(), nexc = (int)ulist[sp].size();
    dexc[sp].assign((size_t)nexc * MSD_EXC, 0);
    for (int e = 0; e < nexc; ++e) {
      const std::vector<int>& u = ulist[sp][e];
      const int k = u[0];
      int* d = &dexc[sp][(size_t)e * MSD_EXC];
      d[0] = k;
      for (int q = 0; q < k; ++q) {
        d[1 + q] = (int)(std::find(hact[sp].begin(), hact[sp].end(), u[1 + q]) - hact[sp].begin());
        d[1 + MSD_KMAX + q] = (int)(std::find(vact.begin(), vact.end(), u[1 + k + q]) - vact.begin());
        d[1 + 2 * MSD_KMAX + q] = u[1 + q];
      }
    }
    // determinants grouped by this spin's excitation, in index order
    std::vector<int> off(nexc + 1, 0), det(n_det);
    for (int I = 0; I < n_det; ++I) ++off[hpair[2 * I + sp] + 1];
    for (int e = 0; e < nexc; ++e) off[e + 1] += off[e];
    std::vector<int> fill(off.begin(), off.end() - 1);
    for (int I = 0; I < n_det; ++I) det[fill[hpair[2 * I + sp]]++] = I;
    AFQ_RET(s->msd_csr_off[sp].alloc(off.size() * sizeof(int)));
    AFQ_RET(s->msd_csr_det[sp].alloc(det.size() * sizeof(int)));
    AFQ_TRY_HIP(hipMemcpyAsync(s->msd_csr_off[sp].p, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->msd_csr_det[sp].p, det.data(), det.size() * sizeof(int), hipMemcpyHostToDevice, st));
    AFQ_RET(s->msd_exc[sp].alloc(dexc[sp].size() * sizeof(int)));
    AFQ_RET(s->msd_hact[sp].alloc((size_t)std::max(no, 1) * sizeof(int)));
    AFQ_TRY_HIP(hipMemcpyAsync(s->msd_exc[sp].p, dexc[sp].data(), dexc[sp].size() * sizeof(int),
                               hipMemcpyHostToDevice, st));
    if (no) AFQ_TRY_HIP(hipMemcpyAsync(s->msd_hact[sp].p, hact[sp].data(), no * sizeof(int), hipMemcpyHostToDevice, st));
  }
  // [C_ref; C_V]^H (nr x M) and Lact[g] = [C_ref; C_V]^H L^g, g = X: h1
  std::vector<double2> cah((size_t)nr * M);
  for (int r = 0; r < nr; ++r) {
    const int col = r < nmax ? r : vact[r - nmax];
    for (int i = 0; i < M; ++i) {
      const double2 c = hC[(size_t)i * M + col];
      cah[(size_t)r * M + i] = make_double2(c.x, -c.y);
    }
  }
  DevBuf cad;
  AFQ_RET(cad.alloc(cah.size() * 16));
  AFQ_TRY_HIP(hipMemcpyAsync(cad.p, cah.data(), cah.size() * 16, hipMemcpyHostToDevice, st));
  AFQ_RET(s->msd_cvh.alloc((size_t)std::max(nv, 1) * M * 16));
  if (nv)
    AFQ_TRY_HIP(hipMemcpyAsync(s->msd_cvh.p, cad.as<double2>() + (size_t)nmax * M, (size_t)nv * M * 16,
                               hipMemcpyDeviceToDevice, st));
  AFQ_RET(s->msd_lact.alloc((size_t)(X + 1) * nr * M * 16));
  {
    GemmArgs<double> g = gemm_args<double>();
    g.m = nr; g.n = M; g.k = M; g.batch = X;
    g.A = cad.as<double>(); g.lda = M; g.cA = true; g.sA = 0;
    g.B = s->chol.as<double>(); g.ldb = M; g.cB = false; g.sB = (long)M * M;
    g.C = s->msd_lact.as<double>(); g.ldc = M; g.cC = true; g.sC = (long)nr * M;
    AFQ_RET(gemm<double>(g, st));
    GemmArgs<double> h = g;
    h.batch = 1;
    h.B = s->h1.as<double>();
    h.C = s->msd_lact.as<double>() + 2L * X * nr * M;
    AFQ_RET(gemm<double>(h, st));
  }
  AFQ_TRY_HIP(hipStreamSynchronize(st));
  if (lds > 64 * 1024)
    AFQ_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(msd_post_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  s->msd_nr = nr;
  s->msd_lds = lds;
  s->msd_n = n_det;
  ++s->version;
  return eri_sync(s);   // a multi-determinant trial has no four-index exchange
}

int msd_alloc_scratch(afq_system s, afq_walkers w) {
  const int nw = w->nw, X = s->X, ntot = s->ntot, nv = s->msd_nv;
  const size_t per_walker = (size_t)(X + 1) * s->msd_nr * ntot * 16;
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(nw, MSD_OMEGA_BUDGET / per_walker));
  const size_t tv = (size_t)nw * std::max(nv, 1) * ntot * 16;
  if (w->msd_tv.bytes < tv) AFQ_RET(w->msd_tv.alloc(tv));
  for (int sp = 0; sp < 2; ++sp) {
    const size_t d0 = (size_t)nw * s->msd_nexc[sp] * 16;
    if (w->msd_d0[sp].bytes < d0) AFQ_RET(w->msd_d0[sp].alloc(d0));
    if (w->msd_S[sp].bytes < d0) AFQ_RET(w->msd_S[sp].alloc(d0));
  }
  const size_t om = (size_t)chunk * per_walker;
  if (w->msd_omega.bytes < om) AFQ_RET(w->msd_omega.alloc(om));
  const size_t num = (size_t)nw * (2 * X + 1) * 16;
  if (w->msd_num.bytes < num) AFQ_RET(w->msd_num.alloc(num));
  if (w->msd_den.bytes < (size_t)nw * 16) AFQ_RET(w->msd_den.alloc((size_t)nw * 16));
  if (w->msd_parts.bytes < (size_t)nw * 48) AFQ_RET(w->msd_parts.alloc((size_t)nw * 48));
  if (w->msd_vbar.bytes < (size_t)nw * X * 16) AFQ_RET(w->msd_vbar.alloc((size_t)nw * X * 16));
  w->msd_chunk = chunk;
  return AFQ_OK;
}

// T_V = C_V^H Theta for every walker (all columns), then det A of every excitation
static int msd_ratios(afq_system s, afq_walkers w, double2* logdet, hipStream_t st) {
  const int M = s->M, ntot = s->ntot, nw = w->nw, nv = s->msd_nv;
  if (nv) {
    GemmArgs<double> g = gemm_args<double>();
    g.m = nv; g.n = ntot; g.k = M; g.batch = nw;
    g.A = s->msd_cvh.as<double>(); g.lda = M; g.cA = true; g.sA = 0;
    g.B = w->theta.as<double>(); g.ldb = M; g.opB = OP_T; g.cB = true; g.sB = (long)ntot * M;
    g.C = w->msd_tv.as<double>(); g.ldc = ntot; g.cC = true; g.sC = (long)nv * ntot;
    AFQ_RET(gemm<double>(g, st));
  }
  for (int sp = 0; sp < 2; ++sp) {
    hipLaunchKernelGGL(msd_ratio_kernel, dim3(ceil_div(s->msd_nexc[sp], 64), nw), dim3(64), 0, st,
                       w->msd_tv.as<double2>(), nv, ntot, s->spin_off(sp), s->msd_exc[sp].as<int>(),
                       s->msd_nexc[sp], w->msd_d0[sp].as<double2>());
    AFQ_TRY_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(msd_den_kernel, dim3(nw), dim3(256), 0, st, s->msd_cconj.as<double2>(), s->msd_pair.as<int>(),
                     s->msd_n, w->msd_d0[0].as<double2>(), s->msd_nexc[0], w->msd_d0[1].as<double2>(),
                     s->msd_nexc[1], w->msd_den.as<double2>(), logdet);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

int msd_overlap(afq_system s, afq_walkers w, double2* logdet, hipStream_t st) {
  AFQ_RET(msd_alloc_scratch(s, w));
  return msd_ratios(s, w, logdet, st);
}

int msd_energy(afq_system s, afq_walkers w, double2* logdet, hipStream_t st) {
  AFQ_RET(msd_alloc_scratch(s, w));
  const int M = s->M, ntot = s->ntot, nw = w->nw, X = s->X, nr = s->msd_nr;
  {
    TraceScope tr(AFQ_PH_MSD_SUMS, st);
    AFQ_RET(msd_ratios(s, w, logdet, st));
    hipLaunchKernelGGL(msd_pairsum_kernel, dim3(nw), dim3(256), 0, st, s->msd_cconj.as<double2>(),
                       s->msd_pair.as<int>(), s->msd_csr_off[0].as<int>(), s->msd_csr_det[0].as<int>(),
                       s->msd_csr_off[1].as<int>(), s->msd_csr_det[1].as<int>(), w->msd_d0[0].as<double2>(),
                       s->msd_nexc[0], w->msd_d0[1].as<double2>(), s->msd_nexc[1], w->msd_S[0].as<double2>(),
                       w->msd_S[1].as<double2>());
    AFQ_TRY_HIP(hipGetLastError());
  }
  MsdPostArgs pa{};
  pa.omega = w->msd_omega.as<double2>();
  pa.tv = w->msd_tv.as<double2>();
  for (int sp = 0; sp < 2; ++sp) {
    pa.exc[sp] = s->msd_exc[sp].as<int>();
    pa.hact[sp] = s->msd_hact[sp].as<int>();
    pa.n[sp] = s->nspin_n(sp);
    pa.off[sp] = s->spin_off(sp);
    pa.no[sp] = s->msd_no[sp];
    pa.nexc[sp] = s->msd_nexc[sp];
    pa.S[sp] = w->msd_S[sp].as<double2>();
  }
  pa.nmax = std::max(s->n_up, s->n_dn);
  pa.nv = s->msd_nv;
  pa.nr = nr;
  pa.ntot = ntot;
  pa.nexc_max = std::max(s->msd_nexc[0], s->msd_nexc[1]);
  pa.pair = s->msd_pair.as<int>();
  pa.cconj = s->msd_cconj.as<double2>();
  pa.ndet = s->msd_n;
  pa.X = X;
  pa.num = w->msd_num.as<double2>();
  for (int w0 = 0; w0 < nw; w0 += w->msd_chunk) {
    const int nc = std::min(w->msd_chunk, nw - w0);
    {
      TraceScope tr(AFQ_PH_MSD_OMEGA, st);
      GemmArgs<double> g = gemm_args<double>();
      g.m = (X + 1) * nr; g.n = nc * ntot; g.k = M;
      g.A = s->msd_lact.as<double>(); g.lda = M; g.cA = true;
      g.B = w->theta.as<double>() + 2L * w0 * ntot * M; g.ldb = M; g.opB = OP_T; g.cB = true;
      g.C = w->msd_omega.as<double>(); g.ldc = (long)nc * ntot; g.cC = true;
      AFQ_RET(gemm<double>(g, st));
    }
    pa.w0 = w0;
    pa.ldo = (long)nc * ntot;
    TraceScope tr(AFQ_PH_MSD_SUMS, st);
    hipLaunchKernelGGL(msd_post_kernel, dim3(X + 1, nc), dim3(256), s->msd_lds, st, pa);
    AFQ_TRY_HIP(hipGetLastError());
  }
  TraceScope tr(AFQ_PH_MSD_SUMS, st);
  hipLaunchKernelGGL(msd_finish_kernel, dim3(nw), dim3(256), 0, st, w->msd_num.as<double2>(),
                     w->msd_den.as<double2>(), X, w->msd_parts.as<double2>(), w->msd_vbar.as<double2>());
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
