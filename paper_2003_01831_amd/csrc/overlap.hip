// The FP64 walker products whose output side is the electron count, on
// v_mfma_f64_16x16x4f64: the two around the overlap inverse (sec:afqmc: the
// mixed Green's function G = W (T^H W)^-1 T^H) and the two of CholeskyQR,
//
//   overlap  S^s_w = T^sH W^s_w          (n x n per walker and spin, contraction over the M basis functions)
//   theta    Theta^s_w = W^s_w (S^s_w)^-1, stored transposed as thetaT[w][off_s + b][k]
//   gram     G^s_w = W^sH_w W^s_w         (upper block triangle, mirrored)
//   qr       Q^s_w = W^s_w (R^s_w)^-1      (the theta kernel, stored in the walker layout)
//
// plus grouped launches of the overlap and theta kernels that walk a work
// table of many walker sets (the systems of a batch).
//
// All have an output side of n <= 128 electrons, which the general tiled GEMM
// pads to 32-row wave tiles (100 -> 128); here every wave owns whole 16-wide
// MFMA blocks over all of n (100 -> 112), the spins share one launch, and the
// contraction runs to its exact length in steps of 4 (no padding of k or j).
// Complex products are four real MFMAs (Re += ar br - ai bi, Im += ar bi +
// ai br); a real trial drops the terms of its zero imaginary part.
//
// Contraction index of MFMA step s in a 16-wide chunk c: lanes of quarter q
// (lane >> 4) supply index 16 c + 4 s + q for both operands; a chunk's
// trailing steps past the end are skipped (uniform branch) and the entries
// past the end inside a step are zero.
#include "common.h"
#include <type_traits>
#include "step_kernels.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mma(d4 c, double a, double b) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

struct OvlArgs {
  const double2* W;      // walker w at W + w * M * ntot; (k, c) at k * ntot + c
  const double* phir;    // real trial: Re T, [M][ntot]; else NULL
  const double2* phi;    // complex trial: T, [M][ntot]
  double2* S;            // (w, s) at S + (2 w + s) * nm2, row-major n_s x n_s
  long nm2;
  int M, ntot, nw;
  int n[2], off[2];
};

// S^s_w[a][j] = sum_k conj(T[k][off + a]) W_w[k][off + j]. The columns (w, j)
// of all walkers of a spin are numbered w n + j and cut into 16-wide blocks
// (a block may straddle two walkers: every lane finds its own); workgroups of
// four waves, one column block each, every wave holding all row blocks a. The
// trial's rows are the operand all waves share: staged through LDS 16 basis
// functions at a time (double buffered, one barrier per chunk); the walker
// fragments come straight from memory, one chunk ahead.
// (workgroup bx of spin sp; 256 threads)
template <int NB, bool CA>
__device__ __forceinline__ void overlap_body(const OvlArgs& g, int bx, int sp) {
  using TE = typename std::conditional<CA, double2, double>::type;
  constexpr int NC = NB * 16, PER = 16 * NC / 256;   // PER = NB
  __shared__ TE As[2][16][NC];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = g.n[sp], off = g.off[sp], M = g.M, ntot = g.ntot;
  const long ncol = (long)g.nw * n;
  if (64L * bx >= ncol) return;   // whole workgroup (the grid covers the larger spin)
  const int r = lane & 15, q = lane >> 4;
  const long col0 = 16L * (4 * bx + wave), col = col0 + r;
  const bool cok = col < ncol;
  const int w = cok ? (int)(col / n) : 0, j = cok ? (int)(col - (long)w * n) : 0;
  const double2* Wl = g.W + (long)w * M * ntot + off + j;   // this lane's column; row k at k * ntot
  const int nchunk = (M + 15) / 16;

  TE st[PER];
  auto fetch_a = [&](int c) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, row = e / NC, a = e - row * NC, k = 16 * c + row;
      const bool ok = k < M && a < n;
      if constexpr (CA) st[u] = ok ? g.phi[(long)k * ntot + off + a] : make_double2(0.0, 0.0);
      else st[u] = ok ? g.phir[(long)k * ntot + off + a] : 0.0;
    }
  };
  auto stash_a = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, row = e / NC, a = e - row * NC;
      As[buf][row][a] = st[u];
    }
  };
  double2 bv[4], nb[4];
  auto fetch_b = [&](int c, double2 (&x)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 16 * c + 4 * s + q;
      x[s] = cok && k < M ? Wl[(long)k * ntot] : make_double2(0.0, 0.0);
    }
  };

  d4 accr[NB], acci[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) accr[i] = acci[i] = d4{0.0, 0.0, 0.0, 0.0};

  fetch_a(0);
  fetch_b(0, bv);
  stash_a(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) {
      fetch_a(c + 1);
      fetch_b(c + 1, nb);
    }
    // MFMA steps of this chunk (none for a column block past the last walker, which only helps stage)
    const int ns = col0 < ncol ? min(4, (M - 16 * c + 3) / 4) : 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s < ns) {
        TE a[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) a[i] = As[buf][4 * s + q][16 * i + r];
        const double br = bv[s].x, bi = bv[s].y;
        if constexpr (CA) {   // A = conj(T): Re a, -Im a
#pragma unroll
          for (int i = 0; i < NB; ++i) accr[i] = mma(accr[i], a[i].x, br);
#pragma unroll
          for (int i = 0; i < NB; ++i) acci[i] = mma(acci[i], a[i].x, bi);
#pragma unroll
          for (int i = 0; i < NB; ++i) accr[i] = mma(accr[i], a[i].y, bi);
#pragma unroll
          for (int i = 0; i < NB; ++i) acci[i] = mma(acci[i], -a[i].y, br);
        } else {
#pragma unroll
          for (int i = 0; i < NB; ++i) accr[i] = mma(accr[i], a[i], br);
#pragma unroll
          for (int i = 0; i < NB; ++i) acci[i] = mma(acci[i], a[i], bi);
        }
      }
    }
    if (c + 1 < nchunk) {
      stash_a(buf ^ 1);
#pragma unroll
      for (int s = 0; s < 4; ++s) bv[s] = nb[s];
    }
    __syncthreads();
  }
  // lane holds rows 16 i + q + 4 t (a) of its column (w, j)
  if (cok) {
    double2* Sw = g.S + (2L * w + sp) * g.nm2 + j;
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int a = 16 * i + q + 4 * t;
        if (a < n) Sw[(long)a * n] = make_double2(accr[i][t], acci[i][t]);
      }
  }
}

template <int NB, bool CA>
__global__ __launch_bounds__(256) void overlap_kernel(OvlArgs g) {
  overlap_body<NB, CA>(g, blockIdx.x, blockIdx.y);
}

// Work table of a grouped launch (walker sets of several systems, one
// electron-block count): workgroup x runs block x - first[t] of task t with
// first[t] <= x < first[t + 1]; passed by value, so a captured graph holds it.
constexpr int OVL_GROUP = 24;
struct OvlGroupArgs {
  OvlArgs g[OVL_GROUP];
  int first[OVL_GROUP + 1];
  int ntask;
};

template <int NB, bool CA>
__global__ __launch_bounds__(256) void overlap_grouped_kernel(OvlGroupArgs G) {
  const int x = blockIdx.x;
  int t = 0;
  while (t + 1 < G.ntask && x >= G.first[t + 1]) ++t;
  const OvlArgs& g = G.g[t];
  overlap_body<NB, CA>(g, x - G.first[t], blockIdx.y);
}

struct ThetaArgs {
  const double2* W;      // as in OvlArgs
  const double2* Sinv;   // (w, s) at Sinv + (2 w + s) * nm2, row-major n_s x n_s
  double2* thetaT;       // walker w at thetaT + w * ntot * M; (off_s + b, k) at (off_s + b) * M + k
                         // (WOUT: in the walker layout, (k, off_s + b) at k * ntot + off_s + b)
  long nm2;
  int M, ntot, nw, nkg, nwv;   // nkg workgroups of nwv waves per walker and spin
  int n[2], off[2];
};

// thetaT[w][off + b][k] = sum_j Sinv[j][b] W[k][off + j]: MFMA rows b (A =
// Sinv^T), columns k (B = W^T), so that a lane quarter stores 16 consecutive
// basis functions. Workgroup: nwv waves over consecutive 16-wide column
// blocks of one walker and spin; each wave holds every row block b against
// its column block. S^-1 is the operand all waves share: staged through LDS
// 16 rows j at a time (double buffered); the W fragments come straight from
// memory, one chunk ahead. Workgroups are numbered so that the nkg of one
// walker land on one XCD (dispatch i goes to XCD i mod 8) and share S^-1 in
// its L2. At NB = 8 the accumulators leave room for 4 waves only. With WOUT
// the product is stored in the walker layout instead (Q = W R^-1 of
// CholeskyQR, R^-1 in place of S^-1).
// (workgroup lin of spin sp; 64 nwv threads)
template <int NB, bool WOUT>
__device__ __forceinline__ void theta_body(const ThetaArgs& g, int lin, int sp) {
  constexpr int NC = NB * 16, PER = 16 * NC / 256;   // staged elements per thread with >= 4 waves
  __shared__ double2 As[2][16][NC];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), nt = blockDim.x;
  const int w = (lin / (8 * g.nkg)) * 8 + (lin & 7), kg = (lin >> 3) % g.nkg;
  const int n = g.n[sp], off = g.off[sp], M = g.M, ntot = g.ntot;
  if (n == 0 || w >= g.nw) return;   // whole workgroup
  const double2* Ww = g.W + (long)w * M * ntot + off;
  const double2* Si = g.Sinv + (2L * w + sp) * g.nm2;
  const int r = lane & 15, q = lane >> 4;
  const int k0 = 16 * (kg * g.nwv + wave), k = k0 + r;   // this lane's column (basis function)
  const bool kcol = k < M;
  const int nchunk = (n + 15) / 16;

  double2 st[PER];
  auto fetch_a = [&](int c) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + nt * u, row = e / NC, col = e - row * NC, j = 16 * c + row;
      st[u] = e < 16 * NC && j < n && col < n ? Si[(long)j * n + col] : make_double2(0.0, 0.0);
    }
  };
  auto stash_a = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + nt * u, row = e / NC, col = e - row * NC;
      if (e < 16 * NC) As[buf][row][col] = st[u];
    }
  };
  double2 bv[4], nb[4];
  auto fetch_b = [&](int c, double2 (&x)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int j = 16 * c + 4 * s + q;
      x[s] = kcol && j < n ? Ww[(long)k * ntot + j] : make_double2(0.0, 0.0);
    }
  };

  d4 accr[NB], acci[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) accr[i] = acci[i] = d4{0.0, 0.0, 0.0, 0.0};

  fetch_a(0);
  fetch_b(0, bv);
  stash_a(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) {
      fetch_a(c + 1);
      fetch_b(c + 1, nb);
    }
    // MFMA steps of this chunk (none for a column block past M, which only helps stage)
    const int ns = k0 < M ? min(4, (n - 16 * c + 3) / 4) : 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s < ns) {
        double2 a[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) a[i] = As[buf][4 * s + q][16 * i + r];
        const double br = bv[s].x, bi = bv[s].y;
#pragma unroll
        for (int i = 0; i < NB; ++i) accr[i] = mma(accr[i], a[i].x, br);
#pragma unroll
        for (int i = 0; i < NB; ++i) acci[i] = mma(acci[i], a[i].x, bi);
#pragma unroll
        for (int i = 0; i < NB; ++i) accr[i] = mma(accr[i], -a[i].y, bi);
#pragma unroll
        for (int i = 0; i < NB; ++i) acci[i] = mma(acci[i], a[i].y, br);
      }
    }
    if (c + 1 < nchunk) {
      stash_a(buf ^ 1);
#pragma unroll
      for (int s = 0; s < 4; ++s) bv[s] = nb[s];
    }
    __syncthreads();
  }
  // lane holds rows 16 i + q + 4 t (b), column k of each block
  if (kcol) {
    double2* Tw = g.thetaT + (long)w * ntot * M + (WOUT ? (long)k * ntot + off : (long)off * M + k);
    const long bstep = WOUT ? 1 : M;
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int b = 16 * i + q + 4 * t;
        if (b < n) Tw[b * bstep] = make_double2(accr[i][t], acci[i][t]);
      }
  }
}

template <int NB, bool WOUT>
__global__ __launch_bounds__(NB == 8 ? 256 : 512) void theta_kernel(ThetaArgs g) {
  theta_body<NB, WOUT>(g, blockIdx.x, blockIdx.y);
}

// grouped Theta launches: as OvlGroupArgs (tasks of one electron-block count
// and one wave count; every task's block count is a multiple of 8, so the
// XCD numbering of each task holds)
constexpr int THETA_GROUP = 24;
struct ThetaGroupArgs {
  ThetaArgs g[THETA_GROUP];
  int first[THETA_GROUP + 1];
  int ntask;
};

template <int NB>
__global__ __launch_bounds__(NB == 8 ? 256 : 512) void theta_grouped_kernel(ThetaGroupArgs G) {
  const int x = blockIdx.x;
  int t = 0;
  while (t + 1 < G.ntask && x >= G.first[t + 1]) ++t;
  const ThetaArgs& g = G.g[t];
  theta_body<NB, false>(g, x - G.first[t], blockIdx.y);
}

struct GramArgs {
  const double2* W;      // as in OvlArgs
  double2* G;            // (w, s) at G + (2 w + s) * nm2, row-major n_s x n_s
  long nm2;
  int M, ntot, nw;
  int n[2], off[2];
};

// Gram matrices G^s_w = W^sH_w W^s_w of CholeskyQR, both spins in one launch:
// workgroup (column group, walker, spin) of four waves, one 16-wide column
// block b each; W's rows (all n_s columns) are staged through LDS 16 basis
// functions at a time and serve both operands. A wave forms only the blocks
// of the upper block triangle (row blocks a <= its column block) and stores
// each off-diagonal one twice, the second time conjugated at the mirrored
// place.
template <int NB>
__global__ __launch_bounds__(256) void gram_kernel(GramArgs g) {
  constexpr int NC = NB * 16, PER = 16 * NC / 256;   // PER = NB
  __shared__ double2 As[2][16][NC];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ncg = (NB + 3) / 4;
  const int cg = blockIdx.x % ncg, w = blockIdx.x / ncg, sp = blockIdx.y;
  const int n = g.n[sp], off = g.off[sp], M = g.M, ntot = g.ntot;
  const int jb = 4 * cg + wave;              // this wave's column block
  if (n == 0 || 64 * cg >= n) return;        // whole workgroup
  const double2* Ww = g.W + (long)w * M * ntot + off;
  const int r = lane & 15, q = lane >> 4;
  const int nchunk = (M + 15) / 16;

  double2 st[PER];
  auto fetch = [&](int c) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, row = e / NC, col = e - row * NC, k = 16 * c + row;
      st[u] = k < M && col < n ? Ww[(long)k * ntot + col] : make_double2(0.0, 0.0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, row = e / NC, col = e - row * NC;
      As[buf][row][col] = st[u];
    }
  };

  d4 accr[NB], acci[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) accr[i] = acci[i] = d4{0.0, 0.0, 0.0, 0.0};
  const bool active = jb < NB && 16 * jb < n;   // wave-uniform

  fetch(0);
  stash(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunk) fetch(c + 1);
    const int ns = active ? min(4, (M - 16 * c + 3) / 4) : 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s < ns) {
        const double2 b = As[buf][4 * s + q][16 * jb + r];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          if (i <= jb) {   // A = conj(W): Re a, -Im a
            const double2 a = As[buf][4 * s + q][16 * i + r];
            accr[i] = mma(accr[i], a.x, b.x);
            acci[i] = mma(acci[i], a.x, b.y);
            accr[i] = mma(accr[i], a.y, b.y);
            acci[i] = mma(acci[i], -a.y, b.x);
          }
        }
      }
    }
    if (c + 1 < nchunk) stash(buf ^ 1);
    __syncthreads();
  }
  if (!active) return;
  // lane holds rows 16 i + q + 4 t (a) of column 16 jb + r (b)
  double2* Gw = g.G + (2L * w + sp) * g.nm2;
  const int b = 16 * jb + r;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i > jb) continue;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int a = 16 * i + q + 4 * t;
      if (a < n && b < n) {
        Gw[(long)a * n + b] = make_double2(accr[i][t], acci[i][t]);
        if (i < jb) Gw[(long)b * n + a] = make_double2(accr[i][t], -acci[i][t]);
      }
    }
  }
}

// waves per theta workgroup: 4 or 8, so that the two waves per SIMD that the
// accumulators leave room for are evenly spread; 8 only where it leaves no
// more column blocks idle
int theta_waves(int nblk) { return ceil_div(nblk, 8) * 8 == ceil_div(nblk, 4) * 4 ? 8 : 4; }

}  // namespace

namespace {
thread_local std::vector<OvlTask>* t_ovl_sink = nullptr;

OvlArgs ovl_args(const OvlTask& t) {
  OvlArgs g{};
  g.W = t.W; g.phir = t.phir; g.phi = t.phi; g.S = t.S; g.nm2 = t.nm2;
  g.M = t.M; g.ntot = t.ntot; g.nw = t.nw;
  for (int s = 0; s < 2; ++s) { g.n[s] = t.n[s]; g.off[s] = t.off[s]; }
  return g;
}
int nb_of(const int n[2]) { return (std::max(n[0], n[1]) + 15) / 16; }
long ovl_blocks(const OvlTask& t) { return ((long)t.nw * std::max(t.n[0], t.n[1]) + 63) / 64; }
}  // namespace

void overlap_defer(std::vector<OvlTask>* sink) { t_ovl_sink = sink; }

int overlap_grouped(const std::vector<OvlTask>& tasks, hipStream_t st) {
  for (int nb = 1; nb <= 8; ++nb)
    for (int ca = 0; ca < 2; ++ca) {
      OvlGroupArgs G{};
      long blocks = 0;
      auto flush = [&]() -> int {
        if (G.ntask == 0) return AFQ_OK;
        AFQ_CHECK(blocks <= INT32_MAX, AFQ_E_INVALID, "overlap: too many workgroups");
        G.first[G.ntask] = (int)blocks;
        const dim3 grid((unsigned)blocks, 2);
#define AFQ_OVLG(NB_)                                                                                      \
  case NB_:                                                                                                \
    if (ca) hipLaunchKernelGGL((overlap_grouped_kernel<NB_, true>), grid, dim3(256), 0, st, G);            \
    else hipLaunchKernelGGL((overlap_grouped_kernel<NB_, false>), grid, dim3(256), 0, st, G);              \
    break;
        switch (nb) { AFQ_OVLG(1) AFQ_OVLG(2) AFQ_OVLG(3) AFQ_OVLG(4) AFQ_OVLG(5) AFQ_OVLG(6) AFQ_OVLG(7) AFQ_OVLG(8) }
#undef AFQ_OVLG
        AFQ_TRY_HIP(hipGetLastError());
        G = OvlGroupArgs{};
        blocks = 0;
        return AFQ_OK;
      };
      for (const OvlTask& t : tasks) {
        if (nb_of(t.n) != nb || (t.phir == nullptr) != (ca != 0) || t.nw <= 0) continue;
        G.g[G.ntask] = ovl_args(t);
        G.first[G.ntask++] = (int)blocks;
        blocks += ovl_blocks(t);
        if (G.ntask == OVL_GROUP) AFQ_RET(flush());
      }
      AFQ_RET(flush());
    }
  return AFQ_OK;
}

int overlap_mfma(const double2* W, const double* phir, const double2* phi, int M, int ntot, int nw, const int n[2],
                 const int off[2], double2* S, long nm2, hipStream_t st) {
  const int nmax = std::max(n[0], n[1]);
  AFQ_CHECK(nmax >= 1 && nmax <= 128 && (phir || phi) && M >= 1 && nw >= 0, AFQ_E_INVALID,
            "overlap: n must be in [1, 128], a trial is needed");
  AFQ_CHECK(nm2 >= (long)nmax * nmax, AFQ_E_INVALID, "overlap: matrix stride < n^2");
  if (nw == 0) return AFQ_OK;
  if (t_ovl_sink) {   // deferred into a grouped launch of many systems
    t_ovl_sink->push_back(OvlTask{W, phir, phi, S, nm2, M, ntot, nw, {n[0], n[1]}, {off[0], off[1]}});
    return AFQ_OK;
  }
  OvlArgs g{};
  g.W = W; g.phir = phir; g.phi = phi; g.S = S; g.nm2 = nm2;
  g.M = M; g.ntot = ntot; g.nw = nw;
  for (int s = 0; s < 2; ++s) { g.n[s] = n[s]; g.off[s] = off[s]; }
  const long blocks = ((long)nw * nmax + 63) / 64;   // four 16-wide column blocks per workgroup
  AFQ_CHECK(blocks <= INT32_MAX, AFQ_E_INVALID, "overlap: too many workgroups");
  const dim3 grid((unsigned)blocks, 2);
  const int nb = (nmax + 15) / 16;
#define AFQ_OVL(NB_)                                                                                   \
  case NB_:                                                                                            \
    if (phir) hipLaunchKernelGGL((overlap_kernel<NB_, false>), grid, dim3(256), 0, st, g);             \
    else hipLaunchKernelGGL((overlap_kernel<NB_, true>), grid, dim3(256), 0, st, g);                   \
    break;
  switch (nb) { AFQ_OVL(1) AFQ_OVL(2) AFQ_OVL(3) AFQ_OVL(4) AFQ_OVL(5) AFQ_OVL(6) AFQ_OVL(7) AFQ_OVL(8) }
#undef AFQ_OVL
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}

namespace {
template <bool WOUT>
int launch_theta(const double2* W, const double2* Sinv, int M, int ntot, int nw, const int n[2], const int off[2],
                 long nm2, double2* out, hipStream_t st) {
  const int nmax = std::max(n[0], n[1]);
  AFQ_CHECK(nmax >= 1 && nmax <= 128 && M >= 1 && nw >= 0, AFQ_E_INVALID, "theta: n must be in [1, 128]");
  AFQ_CHECK(nm2 >= (long)nmax * nmax, AFQ_E_INVALID, "theta: matrix stride < n^2");
  if (nw == 0) return AFQ_OK;
  ThetaArgs g{};
  g.W = W; g.Sinv = Sinv; g.thetaT = out; g.nm2 = nm2;
  g.M = M; g.ntot = ntot; g.nw = nw;
  for (int s = 0; s < 2; ++s) { g.n[s] = n[s]; g.off[s] = off[s]; }
  const int nblk = (M + 15) / 16;
  const int nb = (nmax + 15) / 16;
  g.nwv = nb == 8 ? 4 : theta_waves(nblk);
  g.nkg = ceil_div(nblk, g.nwv);
  // walkers padded to a multiple of 8 (the XCD numbering); the padding returns at once
  const long blocks = (long)ceil_div(nw, 8) * 8 * g.nkg;
  AFQ_CHECK(blocks <= INT32_MAX, AFQ_E_INVALID, "theta: too many workgroups");
  const dim3 grid((unsigned)blocks, 2), block(64 * g.nwv);
#define AFQ_TH(NB_) \
  case NB_: hipLaunchKernelGGL((theta_kernel<NB_, WOUT>), grid, block, 0, st, g); break;
  switch (nb) { AFQ_TH(1) AFQ_TH(2) AFQ_TH(3) AFQ_TH(4) AFQ_TH(5) AFQ_TH(6) AFQ_TH(7) AFQ_TH(8) }
#undef AFQ_TH
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
}  // namespace

int theta_mfma(const double2* W, const double2* Sinv, int M, int ntot, int nw, const int n[2], const int off[2],
               long nm2, double2* thetaT, hipStream_t st) {
  return launch_theta<false>(W, Sinv, M, ntot, nw, n, off, nm2, thetaT, st);
}

int theta_grouped(const std::vector<ThetaTask>& tasks, hipStream_t st) {
  for (const ThetaTask& t : tasks) {
    const int nmax = std::max(t.n[0], t.n[1]);
    AFQ_CHECK(nmax >= 1 && nmax <= 128 && t.M >= 1 && t.nm2 >= (long)nmax * nmax, AFQ_E_INVALID,
              "theta: n must be in [1, 128]");
  }
  for (int nb = 1; nb <= 8; ++nb)
    for (int nwv = 4; nwv <= 8; nwv += 4) {
      ThetaGroupArgs G{};
      long blocks = 0;
      auto flush = [&]() -> int {
        if (G.ntask == 0) return AFQ_OK;
        AFQ_CHECK(blocks <= INT32_MAX, AFQ_E_INVALID, "theta: too many workgroups");
        G.first[G.ntask] = (int)blocks;
        const dim3 grid((unsigned)blocks, 2), block(64 * nwv);
#define AFQ_THG(NB_) \
  case NB_: hipLaunchKernelGGL((theta_grouped_kernel<NB_>), grid, block, 0, st, G); break;
        switch (nb) { AFQ_THG(1) AFQ_THG(2) AFQ_THG(3) AFQ_THG(4) AFQ_THG(5) AFQ_THG(6) AFQ_THG(7) AFQ_THG(8) }
#undef AFQ_THG
        AFQ_TRY_HIP(hipGetLastError());
        G = ThetaGroupArgs{};
        blocks = 0;
        return AFQ_OK;
      };
      for (const ThetaTask& t : tasks) {
        if (t.nw <= 0 || nb_of(t.n) != nb) continue;
        const int nblk = (t.M + 15) / 16;
        const int v = nb == 8 ? 4 : theta_waves(nblk);
        if (v != nwv) continue;
        ThetaArgs g{};
        g.W = t.W; g.Sinv = t.Sinv; g.thetaT = t.thetaT; g.nm2 = t.nm2;
        g.M = t.M; g.ntot = t.ntot; g.nw = t.nw;
        for (int s = 0; s < 2; ++s) { g.n[s] = t.n[s]; g.off[s] = t.off[s]; }
        g.nwv = v;
        g.nkg = ceil_div(nblk, v);
        G.g[G.ntask] = g;
        G.first[G.ntask++] = (int)blocks;
        blocks += (long)ceil_div(t.nw, 8) * 8 * g.nkg;   // a multiple of 8: every task's XCD numbering holds
        if (G.ntask == THETA_GROUP) AFQ_RET(flush());
      }
      AFQ_RET(flush());
    }
  return AFQ_OK;
}

int qr_apply_mfma(const double2* W, const double2* Rinv, int M, int ntot, int nw, const int n[2], const int off[2],
                  long nm2, double2* Q, hipStream_t st) {
  AFQ_CHECK(Q != W, AFQ_E_INVALID, "qr: the output must not overwrite the input");
  return launch_theta<true>(W, Rinv, M, ntot, nw, n, off, nm2, Q, st);
}

int gram_mfma(const double2* W, int M, int ntot, int nw, const int n[2], const int off[2], double2* G, long nm2,
              hipStream_t st) {
  const int nmax = std::max(n[0], n[1]);
  AFQ_CHECK(nmax >= 1 && nmax <= 128 && M >= 1 && nw >= 0, AFQ_E_INVALID, "gram: n must be in [1, 128]");
  AFQ_CHECK(nm2 >= (long)nmax * nmax, AFQ_E_INVALID, "gram: matrix stride < n^2");
  if (nw == 0) return AFQ_OK;
  GramArgs g{};
  g.W = W; g.G = G; g.nm2 = nm2;
  g.M = M; g.ntot = ntot; g.nw = nw;
  for (int s = 0; s < 2; ++s) { g.n[s] = n[s]; g.off[s] = off[s]; }
  const int nb = (nmax + 15) / 16, ncg = (nb + 3) / 4;
  AFQ_CHECK((long)nw * ncg <= INT32_MAX, AFQ_E_INVALID, "gram: too many workgroups");
  const dim3 grid((unsigned)(nw * ncg), 2);
#define AFQ_GR(NB_) \
  case NB_: hipLaunchKernelGGL((gram_kernel<NB_>), grid, dim3(256), 0, st, g); break;
  switch (nb) { AFQ_GR(1) AFQ_GR(2) AFQ_GR(3) AFQ_GR(4) AFQ_GR(5) AFQ_GR(6) AFQ_GR(7) AFQ_GR(8) }
#undef AFQ_GR
  AFQ_TRY_HIP(hipGetLastError());
  return AFQ_OK;
}
