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
// Work per step: one FP64 MFMA GEMM per spin over (X + 1) operators (L^g and
// h1) and the reference plus active-virtual rows, then one workgroup per
// (walker, operator) for the small products and the determinant sums.
#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <vector>
#include "common.h"
#include "step_kernels.h"
#include "trace.h"

constexpr int MSD_MAX_N = 64;     // electrons per spin
constexpr int MSD_MAX_NO = 16;    // active holes per spin
constexpr int MSD_MAX_NV = 32;    // active virtual orbitals per spin
constexpr int MSD_MAX_EXC = 256;  // distinct excitations per spin
constexpr size_t MSD_OMEGA_BUDGET = size_t(2) << 30;   // bytes of Omega per spin and walker chunk

// ---------------------------------------------------------------------------
// small determinants: rows/columns of the k x k block not in the skip masks
// ---------------------------------------------------------------------------
__device__ inline double2 det2(double2 a, double2 b, double2 c, double2 d) { return csub(cmul(a, d), cmul(b, c)); }

__device__ double2 sub_det(const double2 (&A)[MSD_KMAX][MSD_KMAX], int k, unsigned rskip, unsigned cskip) {
  int r[MSD_KMAX], c[MSD_KMAX], m = 0, mc = 0;
  for (int i = 0; i < k; ++i) {
    if (!((rskip >> i) & 1)) r[m++] = i;
    if (!((cskip >> i) & 1)) c[mc++] = i;
  }
  if (m == 0) return make_double2(1.0, 0.0);
  if (m == 1) return A[r[0]][c[0]];
  if (m == 2) return det2(A[r[0]][c[0]], A[r[0]][c[1]], A[r[1]][c[0]], A[r[1]][c[1]]);
  // m = 3 or 4: expansion along the first remaining row
  double2 s = make_double2(0.0, 0.0);
  for (int j = 0; j < m; ++j) {
    double2 minor;
    if (m == 3) {
      int cc[2], q = 0;
      for (int t = 0; t < 3; ++t)
        if (t != j) cc[q++] = c[t];
      minor = det2(A[r[1]][cc[0]], A[r[1]][cc[1]], A[r[2]][cc[0]], A[r[2]][cc[1]]);
    } else {
      int cc[3], q = 0;
      for (int t = 0; t < 4; ++t)
        if (t != j) cc[q++] = c[t];
      const double2 m0 = det2(A[r[2]][cc[1]], A[r[2]][cc[2]], A[r[3]][cc[1]], A[r[3]][cc[2]]);
      const double2 m1 = det2(A[r[2]][cc[0]], A[r[2]][cc[2]], A[r[3]][cc[0]], A[r[3]][cc[2]]);
      const double2 m2 = det2(A[r[2]][cc[0]], A[r[2]][cc[1]], A[r[3]][cc[0]], A[r[3]][cc[1]]);
      minor = cadd(csub(cmul(A[r[1]][cc[0]], m0), cmul(A[r[1]][cc[1]], m1)), cmul(A[r[1]][cc[2]], m2));
    }
    const double2 term = cmul(A[r[0]][c[j]], minor);
    s = (j & 1) ? csub(s, term) : cadd(s, term);
  }
  return s;
}

// pair index of rows (q1 < q2) among k rows, in the order (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)
__device__ inline int pair_index(int q1, int q2) {
  return q1 == 0 ? q2 - 1 : (q1 == 1 ? q2 + 1 : 5);
}

// ---------------------------------------------------------------------------
// per (walker, excitation): A = T_V[p][h], det A, first-order cofactors
// cof1[q][r] = (-1)^(q+r) minor(q; r) and second-order cofactors
// cof2[(q1,q2)][(r1,r2)] = (-1)^(q1+q2+r1+r2) minor({q1,q2}; {r1,r2})
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void msd_cof_kernel(const double2* __restrict__ tv, int n, int nv,
                                                     const int* __restrict__ exc, const int* __restrict__ hact,
                                                     int nexc, double2* __restrict__ cof, int det_only) {
  const int e = blockIdx.x * 64 + threadIdx.x, w = blockIdx.y;
  if (e >= nexc) return;
  const int* ex = exc + e * MSD_EXC;
  const int k = ex[0];
  const double2* T = tv + (long)w * nv * n;
  double2 A[MSD_KMAX][MSD_KMAX];
  for (int q = 0; q < MSD_KMAX; ++q)
    for (int r = 0; r < MSD_KMAX; ++r)
      A[q][r] = (q < k && r < k) ? T[ex[1 + MSD_KMAX + q] * n + hact[ex[1 + r]]] : make_double2(0.0, 0.0);
  double2* out = cof + ((long)w * nexc + e) * MSD_NCOF;
  out[0] = sub_det(A, k, 0u, 0u);
  if (det_only) return;
  for (int q = 0; q < MSD_KMAX; ++q)
    for (int r = 0; r < MSD_KMAX; ++r) {
      double2 v = make_double2(0.0, 0.0);
      if (q < k && r < k) {
        v = sub_det(A, k, 1u << q, 1u << r);
        if ((q + r) & 1) v = make_double2(-v.x, -v.y);
      }
      out[1 + q * MSD_KMAX + r] = v;
    }
  for (int q1 = 0; q1 < MSD_KMAX; ++q1)
    for (int q2 = q1 + 1; q2 < MSD_KMAX; ++q2)
      for (int r1 = 0; r1 < MSD_KMAX; ++r1)
        for (int r2 = r1 + 1; r2 < MSD_KMAX; ++r2) {
          double2 v = make_double2(0.0, 0.0);
          if (q2 < k && r2 < k) {
            v = sub_det(A, k, (1u << q1) | (1u << q2), (1u << r1) | (1u << r2));
            if ((q1 + q2 + r1 + r2) & 1) v = make_double2(-v.x, -v.y);
          }
          out[1 + MSD_KMAX * MSD_KMAX + pair_index(q1, q2) * 6 + pair_index(r1, r2)] = v;
        }
}

// ---------------------------------------------------------------------------
// per walker: den = sum_I conj(c_I) R_I(up) R_I(down); logdet[2w] += log den
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_den_kernel(const double2* __restrict__ cconj, const int* __restrict__ pair,
                                                      int ndet, const double2* __restrict__ cof0, int nexc0,
                                                      const double2* __restrict__ cof1, int nexc1,
                                                      double2* __restrict__ den, double2* __restrict__ logdet) {
  const int w = blockIdx.x, t = threadIdx.x;
  __shared__ double2 red[256];
  double2 acc = make_double2(0.0, 0.0);
  for (int I = t; I < ndet; I += 256) {
    const double2 ru = cof0[((long)w * nexc0 + pair[2 * I]) * MSD_NCOF];
    const double2 rd = cof1[((long)w * nexc1 + pair[2 * I + 1]) * MSD_NCOF];
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
// one workgroup per (walker of the chunk, operator g in [0, X]): both spins'
// small products, per-excitation polynomials, then the determinant sums
// ---------------------------------------------------------------------------
struct MsdPostArgs {
  const double2* omega[2];   // chunk x (X+1) x (n + nv) x n
  const double2* tv[2];      // nw x nv x n
  const double2* cof[2];     // nw x nexc x NCOF
  const int* exc[2];
  const int* hact[2];
  int n[2], nv[2], no[2], nexc[2];
  const int* pair;
  const double2* cconj;
  int ndet, X, w0;
  double2* num;              // nw x (2X + 1)
};

__global__ __launch_bounds__(256) void msd_post_kernel(MsdPostArgs a) {
  const int g = blockIdx.x, wl = blockIdx.y, w = a.w0 + wl, t = threadIdx.x;
  __shared__ double2 P[MSD_MAX_N * MSD_MAX_NO];
  __shared__ double2 Q[MSD_MAX_N * MSD_MAX_NO];
  __shared__ double2 Y1[MSD_MAX_NV * MSD_MAX_NO];
  __shared__ double2 Y2[MSD_MAX_NV * MSD_MAX_NO];
  __shared__ double2 N1[2][MSD_MAX_EXC];
  __shared__ double2 P2[2][MSD_MAX_EXC];
  __shared__ double2 red[2][256];
  for (int sp = 0; sp < 2; ++sp) {
    const int n = a.n[sp], nv = a.nv[sp], no = a.no[sp], nr = n + nv;
    const double2* om = a.omega[sp] + ((long)wl * (a.X + 1) + g) * nr * n;
    const double2* T = a.tv[sp] + (long)w * nv * n;
    const int* hact = a.hact[sp];
    // traces of the reference block: t0 = tr Omega0, q0 = tr Omega0^2
    double2 t0 = make_double2(0.0, 0.0), q0 = make_double2(0.0, 0.0);
    for (int i = t; i < n; i += 256) t0 = cadd(t0, om[i * n + i]);
    for (int e = t; e < n * n; e += 256) {
      const int i = e / n, j = e - i * n;
      q0 = cadd(q0, cmul(om[i * n + j], om[j * n + i]));
    }
    red[0][t] = t0;
    red[1][t] = q0;
    // P[l][hh] = Omega0[l][h_hh]
    for (int e = t; e < n * no; e += 256) {
      const int l = e / no, hh = e - l * no;
      P[e] = om[l * n + hact[hh]];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) {
        red[0][t] = cadd(red[0][t], red[0][t + s]);
        red[1][t] = cadd(red[1][t], red[1][t + s]);
      }
      __syncthreads();
    }
    t0 = red[0][0];
    q0 = red[1][0];
    // Q = Omega0 P = (Omega0^2)[:, h]
    for (int e = t; e < n * no; e += 256) {
      const int l = e / no, hh = e - l * no;
      double2 s = make_double2(0.0, 0.0);
      for (int j = 0; j < n; ++j) s = cadd(s, cmul(om[l * n + j], P[j * no + hh]));
      Q[e] = s;
    }
    __syncthreads();
    // Y1 = Omega_V[:, h] - T_V P ;  Y2 = -Omega_V P + T_V Q
    for (int e = t; e < nv * no; e += 256) {
      const int v = e / no, hh = e - v * no;
      const double2* ov = om + (long)(n + v) * n;
      double2 y1 = ov[hact[hh]], y2 = make_double2(0.0, 0.0);
      for (int l = 0; l < n; ++l) {
        const double2 tvl = T[v * n + l];
        y1 = csub(y1, cmul(tvl, P[l * no + hh]));
        y2 = cadd(y2, csub(cmul(tvl, Q[l * no + hh]), cmul(ov[l], P[l * no + hh])));
      }
      Y1[e] = y1;
      Y2[e] = y2;
    }
    __syncthreads();
    // per excitation: d1 = sum cof1 Y1, d2 = sum cof1 Y2 + sum cof2 (2 x 2 minors of Y1)
    const double2* cof = a.cof[sp] + (long)w * a.nexc[sp] * MSD_NCOF;
    for (int e = t; e < a.nexc[sp]; e += 256) {
      const int* ex = a.exc[sp] + e * MSD_EXC;
      const int k = ex[0];
      const double2* cf = cof + (long)e * MSD_NCOF;
      double2 y1[MSD_KMAX][MSD_KMAX];
      double2 d1 = make_double2(0.0, 0.0), d2 = make_double2(0.0, 0.0);
      for (int q = 0; q < k; ++q)
        for (int r = 0; r < k; ++r) {
          const int idx = ex[1 + MSD_KMAX + q] * no + ex[1 + r];
          y1[q][r] = Y1[idx];
          const double2 c1 = cf[1 + q * MSD_KMAX + r];
          d1 = cadd(d1, cmul(c1, Y1[idx]));
          d2 = cadd(d2, cmul(c1, Y2[idx]));
        }
      for (int q1 = 0; q1 < k; ++q1)
        for (int q2 = q1 + 1; q2 < k; ++q2)
          for (int r1 = 0; r1 < k; ++r1)
            for (int r2 = r1 + 1; r2 < k; ++r2) {
              const double2 m = det2(y1[q1][r1], y1[q1][r2], y1[q2][r1], y1[q2][r2]);
              d2 = cadd(d2, cmul(m, cf[1 + MSD_KMAX * MSD_KMAX + pair_index(q1, q2) * 6 + pair_index(r1, r2)]));
            }
      const double2 d0 = cf[0];
      N1[sp][e] = cadd(d1, cmul(t0, d0));
      // P2 = 2 d2 + 2 t0 d1 + (t0^2 - q0) d0
      P2[sp][e] = cadd(cadd(cscale(d2, 2.0), cscale(cmul(t0, d1), 2.0)), cmul(csub(cmul(t0, t0), q0), d0));
    }
    __syncthreads();
  }
  // determinant sums
  double2 av = make_double2(0.0, 0.0), ae = make_double2(0.0, 0.0);
  const double2* cu = a.cof[0] + (long)w * a.nexc[0] * MSD_NCOF;
  const double2* cd = a.cof[1] + (long)w * a.nexc[1] * MSD_NCOF;
  for (int I = t; I < a.ndet; I += 256) {
    const int eu = a.pair[2 * I], ed = a.pair[2 * I + 1];
    const double2 c = a.cconj[I];
    const double2 ru = cu[(long)eu * MSD_NCOF], rd = cd[(long)ed * MSD_NCOF];
    const double2 n1u = N1[0][eu], n1d = N1[1][ed];
    av = cadd(av, cmul(c, cadd(cmul(n1u, rd), cmul(ru, n1d))));
    const double2 two = cadd(cadd(cmul(P2[0][eu], rd), cmul(ru, P2[1][ed])), cscale(cmul(n1u, n1d), 2.0));
    ae = cadd(ae, cmul(c, cscale(two, 0.5)));
  }
  red[0][t] = av;
  red[1][t] = ae;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      red[0][t] = cadd(red[0][t], red[0][t + s]);
      red[1][t] = cadd(red[1][t], red[1][t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    double2* out = a.num + (long)w * (2 * a.X + 1);
    if (g < a.X) {
      out[g] = red[0][0];
      out[a.X + g] = red[1][0];
    } else {
      out[2 * a.X] = red[0][0];
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
int msd_set(afq_system s, const double* C, int n_det, const double* coeffs, const int32_t* exc) {
  hipStream_t st = s->stream;
  const int M = s->M, X = s->X;
  if (n_det == 0) {
    s->msd_n = 0;
    return AFQ_OK;
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
  // excitations: validate, collect active holes / virtuals and distinct excitations per spin
  std::set<std::vector<int>> seen;
  std::vector<int> hpair((size_t)2 * n_det);
  std::vector<std::vector<int>> hact(2), vact(2);
  std::vector<std::map<std::vector<int>, int>> uniq(2);
  std::vector<std::vector<std::vector<int>>> ulist(2);
  for (int I = 0; I < n_det; ++I) {
    std::vector<int> key;
    for (int sp = 0; sp < 2; ++sp) {
      const int32_t* r = exc + ((size_t)I * 2 + sp) * MSD_EXC;
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
      }
      key.insert(key.end(), e.begin(), e.end());
      // the occupation set decides orthogonality; the slot pairing only fixes the sign
      auto it = uniq[sp].find(e);
      if (it == uniq[sp].end()) {
        it = uniq[sp].emplace(e, (int)ulist[sp].size()).first;
        ulist[sp].push_back(e);
      }
      hpair[2 * I + sp] = it->second;
      for (int q = 0; q < k; ++q) {
        if (std::find(hact[sp].begin(), hact[sp].end(), e[1 + q]) == hact[sp].end()) hact[sp].push_back(e[1 + q]);
        if (std::find(vact[sp].begin(), vact[sp].end(), e[1 + k + q]) == vact[sp].end())
          vact[sp].push_back(e[1 + k + q]);
      }
    }
    // distinct occupation sets: compare sorted holes and particles per spin
    std::vector<int> occ;
    for (int sp = 0; sp < 2; ++sp) {
      const std::vector<int>& e = ulist[sp][hpair[2 * I + sp]];
      const int k = e[0];
      std::vector<int> h(e.begin() + 1, e.begin() + 1 + k), p(e.begin() + 1 + k, e.end());
      std::sort(h.begin(), h.end());
      std::sort(p.begin(), p.end());
      occ.push_back(-1 - sp);
      occ.insert(occ.end(), h.begin(), h.end());
      occ.push_back(-10 - sp);
      occ.insert(occ.end(), p.begin(), p.end());
    }
    AFQ_CHECK(seen.insert(occ).second, AFQ_E_INVALID,
              "afq_system_set_msd: two determinants have the same occupation (the expansion must be orthogonal)");
  }
  for (int sp = 0; sp < 2; ++sp) {
    AFQ_CHECK((int)hact[sp].size() <= MSD_MAX_NO && (int)vact[sp].size() <= MSD_MAX_NV &&
                  (int)ulist[sp].size() <= MSD_MAX_EXC,
              AFQ_E_UNSUPPORTED,
              "afq_system_set_msd: at most 16 active holes, 32 active virtuals and 256 distinct excitations per spin");
    std::sort(hact[sp].begin(), hact[sp].end());
    std::sort(vact[sp].begin(), vact[sp].end());
  }
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
  std::vector<std::vector<double2>> cvh(2);
  for (int sp = 0; sp < 2; ++sp) {
    const int n = s->nspin_n(sp), off = s->spin_off(sp);
    const int nv = (int)vact[sp].size(), no = (int)hact[sp].size(), nexc = (int)ulist[sp].size();
    dexc[sp].assign((size_t)nexc * MSD_EXC, 0);
    for (int e = 0; e < nexc; ++e) {
      const std::vector<int>& u = ulist[sp][e];
      const int k = u[0];
      dexc[sp][(size_t)e * MSD_EXC] = k;
      for (int q = 0; q < k; ++q) {
        dexc[sp][(size_t)e * MSD_EXC + 1 + q] =
            (int)(std::find(hact[sp].begin(), hact[sp].end(), u[1 + q]) - hact[sp].begin());
        dexc[sp][(size_t)e * MSD_EXC + 1 + MSD_KMAX + q] =
            (int)(std::find(vact[sp].begin(), vact[sp].end(), u[1 + k + q]) - vact[sp].begin());
      }
    }
    cvh[sp].resize((size_t)std::max(nv, 1) * M);
    for (int v = 0; v < nv; ++v)
      for (int i = 0; i < M; ++i) {
        const double2 c = hC[(size_t)i * M + vact[sp][v]];
        cvh[sp][(size_t)v * M + i] = make_double2(c.x, -c.y);
      }
    AFQ_RET(s->msd_exc[sp].alloc(dexc[sp].size() * sizeof(int)));
    AFQ_RET(s->msd_hact[sp].alloc((size_t)std::max(no, 1) * sizeof(int)));
    AFQ_RET(s->msd_cvh[sp].alloc(cvh[sp].size() * 16));
    AFQ_TRY_HIP(hipMemcpyAsync(s->msd_exc[sp].p, dexc[sp].data(), dexc[sp].size() * sizeof(int),
                               hipMemcpyHostToDevice, st));
    if (no) AFQ_TRY_HIP(hipMemcpyAsync(s->msd_hact[sp].p, hact[sp].data(), no * sizeof(int), hipMemcpyHostToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->msd_cvh[sp].p, cvh[sp].data(), cvh[sp].size() * 16, hipMemcpyHostToDevice, st));
    // Lact[g] = [T^H L^g ; C_V^H L^g] (rows n + nv), g = X: h1
    const int nr = n + nv;
    AFQ_RET(s->msd_lact[sp].alloc((size_t)(X + 1) * nr * M * 16));
    AFQ_TRY_HIP(hipMemcpy2DAsync(s->msd_lact[sp].p, (size_t)nr * M * 16, s->Lt.as<double2>() + (size_t)off * M,
                                 (size_t)s->ntot * M * 16, (size_t)n * M * 16, X, hipMemcpyDeviceToDevice, st));
    AFQ_TRY_HIP(hipMemcpyAsync(s->msd_lact[sp].as<double2>() + (size_t)X * nr * M, s->ht.as<double2>() + (size_t)off * M,
                               (size_t)n * M * 16, hipMemcpyDeviceToDevice, st));
    if (nv) {
      GemmArgs<double> g = gemm_args<double>();
      g.m = nv; g.n = M; g.k = M; g.batch = X;
      g.A = s->msd_cvh[sp].as<double>(); g.lda = M; g.cA = true; g.sA = 0;
      g.B = s->chol.as<double>(); g.ldb = M; g.cB = false; g.sB = (long)M * M;
      g.C = s->msd_lact[sp].as<double>() + 2L * n * M; g.ldc = M; g.cC = true; g.sC = (long)nr * M;
      AFQ_RET(gemm<double>(g, st));
      GemmArgs<double> h = g;
      h.batch = 1;
      h.B = s->h1.as<double>();
      h.C = s->msd_lact[sp].as<double>() + 2L * ((long)X * nr + n) * M;
      AFQ_RET(gemm<double>(h, st));
    }
    s->msd_no[sp] = no;
    s->msd_nv[sp] = nv;
    s->msd_nexc[sp] = nexc;
  }
  AFQ_TRY_HIP(hipStreamSynchronize(st));
  s->msd_n = n_det;
  return AFQ_OK;
}

int msd_alloc_scratch(afq_system s, afq_walkers w) {
  const int nw = w->nw, X = s->X;
  size_t per_walker = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const int n = s->nspin_n(sp), nv = s->msd_nv[sp];
    per_walker = std::max(per_walker, (size_t)(X + 1) * (n + nv) * n * 16);
  }
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(nw, MSD_OMEGA_BUDGET / per_walker));
  for (int sp = 0; sp < 2; ++sp) {
    const int n = s->nspin_n(sp), nv = s->msd_nv[sp];
    const size_t tv = (size_t)nw * std::max(nv, 1) * n * 16;
    const size_t cof = (size_t)nw * s->msd_nexc[sp] * MSD_NCOF * 16;
    const size_t om = (size_t)chunk * (X + 1) * (n + nv) * n * 16;
    if (w->msd_tv[sp].bytes < tv) AFQ_RET(w->msd_tv[sp].alloc(tv));
    if (w->msd_cof[sp].bytes < cof) AFQ_RET(w->msd_cof[sp].alloc(cof));
    if (w->msd_omega[sp].bytes < om) AFQ_RET(w->msd_omega[sp].alloc(om));
  }
  const size_t num = (size_t)nw * (2 * X + 1) * 16;
  if (w->msd_num.bytes < num) AFQ_RET(w->msd_num.alloc(num));
  if (w->msd_den.bytes < (size_t)nw * 16) AFQ_RET(w->msd_den.alloc((size_t)nw * 16));
  if (w->msd_parts.bytes < (size_t)nw * 48) AFQ_RET(w->msd_parts.alloc((size_t)nw * 48));
  if (w->msd_vbar.bytes < (size_t)nw * X * 16) AFQ_RET(w->msd_vbar.alloc((size_t)nw * X * 16));
  w->msd_chunk = chunk;
  return AFQ_OK;
}

// T_V = C_V^H Theta for every walker and spin, then det A (and cofactors)
static int msd_ratios(afq_system s, afq_walkers w, bool det_only, double2* logdet, hipStream_t st) {
  const int M = s->M, ntot = s->ntot, nw = w->nw;
  for (int sp = 0; sp < 2; ++sp) {
    const int n = s->nspin_n(sp), off = s->spin_off(sp), nv = s->msd_nv[sp];
    if (nv) {
      GemmArgs<double> g = gemm_args<double>();
      g.m = nv; g.n = n; g.k = M; g.batch = nw;
      g.A = s->msd_cvh[sp].as<double>(); g.lda = M; g.cA = true; g.sA = 0;
      g.B = w->theta.as<double>() + 2L * off * M; g.ldb = M; g.opB = OP_T; g.cB = true; g.sB = (long)ntot * M;
      g.C = w->msd_tv[sp].as<double>(); g.ldc = n; g.cC = true; g.sC = (long)nv * n;
      AFQ_RET(gemm<double>(g, st));
    }
    hipLaunchKernelGGL(msd_cof_kernel, dim3(ceil_div(s->msd_nexc[sp], 64), nw), dim3(64), 0, st,
                       w->msd_tv[sp].as<double2>(), n, nv, s->msd_exc[sp].as<int>(), s->msd_hact[sp].as<int>(),
                       s->msd_nexc[sp], w->msd_cof[sp].as<double2>(), det_only ? 1 : 0);
    AFQ_TRY_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(msd_den_kernel, dim3(nw), dim3(256), 0, st, s->msd_cconj.as<double2>(), s->msd_pair.as<int>(),
                     s->msd_n, w->msd_cof[0].as<double2>(), s->msd_nexc[0], w->msd_cof[1].as<double2>(),
                     s->msd_nexc[1], w->msd_den.as<double2>(), logdet);
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

int msd_overlap(afq_system s, afq_walkers w, double2* logdet, hipStream_t st) {
  AFQ_RET(msd_alloc_scratch(s, w));
  return msd_ratios(s, w, true, logdet, st);
}

int msd_energy(afq_system s, afq_walkers w, double2* logdet, hipStream_t st) {
  AFQ_RET(msd_alloc_scratch(s, w));
  const int M = s->M, ntot = s->ntot, nw = w->nw, X = s->X;
  {
    TraceScope tr(AFQ_PH_PACK, st);
    AFQ_RET(msd_ratios(s, w, false, logdet, st));
  }
  TraceScope tr(AFQ_PH_EXCHANGE, st);
  MsdPostArgs pa{};
  for (int sp = 0; sp < 2; ++sp) {
    pa.omega[sp] = w->msd_omega[sp].as<double2>();
    pa.tv[sp] = w->msd_tv[sp].as<double2>();
    pa.cof[sp] = w->msd_cof[sp].as<double2>();
    pa.exc[sp] = s->msd_exc[sp].as<int>();
    pa.hact[sp] = s->msd_hact[sp].as<int>();
    pa.n[sp] = s->nspin_n(sp);
    pa.nv[sp] = s->msd_nv[sp];
    pa.no[sp] = s->msd_no[sp];
    pa.nexc[sp] = s->msd_nexc[sp];
  }
  pa.pair = s->msd_pair.as<int>();
  pa.cconj = s->msd_cconj.as<double2>();
  pa.ndet = s->msd_n;
  pa.X = X;
  pa.num = w->msd_num.as<double2>();
  for (int w0 = 0; w0 < nw; w0 += w->msd_chunk) {
    const int nc = std::min(w->msd_chunk, nw - w0);
    for (int sp = 0; sp < 2; ++sp) {
      const int n = s->nspin_n(sp), off = s->spin_off(sp), nr = n + s->msd_nv[sp];
      GemmArgs<double> g = gemm_args<double>();
      g.m = (X + 1) * nr; g.n = n; g.k = M; g.batch = nc;
      g.A = s->msd_lact[sp].as<double>(); g.lda = M; g.cA = true; g.sA = 0;
      g.B = w->theta.as<double>() + 2L * ((long)w0 * ntot + off) * M; g.ldb = M; g.opB = OP_T; g.cB = true;
      g.sB = (long)ntot * M;
      g.C = w->msd_omega[sp].as<double>(); g.ldc = n; g.cC = true; g.sC = (long)(X + 1) * nr * n;
      AFQ_RET(gemm<double>(g, st));
    }
    pa.w0 = w0;
    hipLaunchKernelGGL(msd_post_kernel, dim3(X + 1, nc), dim3(256), 0, st, pa);
    AFQ_TRY_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(msd_finish_kernel, dim3(nw), dim3(256), 0, st, w->msd_num.as<double2>(),
                     w->msd_den.as<double2>(), X, w->msd_parts.as<double2>(), w->msd_vbar.as<double2>());
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
