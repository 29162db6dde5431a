// Building blocks of the MFMA kernels that stream both operands through a
// three-stage LDS ring filled by direct global->LDS loads (split-BF16x3 and
// FP32 contractions):
//
//   * operands are packed chunk-major in HBM: 64 bytes per row and chunk (32
//     BF16 or 16 FP32 contraction elements), all rows of chunk 0, then chunk 1,
//     ..., split BF16 with separate hi and lo planes;
//   * one LDS stage holds four regions (A hi, A lo, B hi, B lo) of REG bytes;
//     rows are 64 bytes whose 16-byte pieces are XOR-swizzled, so fragment
//     reads (16 bytes per lane) spread over the banks;
//   * bf3_stream runs the chunk loop of a wave's TA x TB block of 16 x 16
//     tiles as hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with FP32
//     accumulators and the fragments in registers; mma_f32 multiplies one
//     FP32 chunk on v_mfma_f32_16x16x4f32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ring {

typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((address_space(3))) unsigned char lds_t;

constexpr int KC = 32;              // contraction elements per chunk (bf16)
constexpr int ROWB = KC * 2;        // bytes per LDS row per plane (one chunk of one row)
constexpr int CPR = ROWB / 16;      // 16-byte pieces per row

// XOR swizzle of the 16-byte pieces of a 64-byte row (an involution)
__device__ inline int swz(int row, int c) { return c ^ ((row >> 1) & 3); }

__device__ inline uint4 lds16(const unsigned char* p) { return *reinterpret_cast<const uint4*>(p); }

// The bf16 fragment of lane (lr, lq) of a 16 x 32 tile starting at `row`: row
// row + lr, elements 8 lq .. 8 lq + 7, read from an LDS-qualified plane
// pointer (a ds_read_b128 whatever the caller's pointer arithmetic hides from
// address-space inference)
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
typedef __attribute__((address_space(3))) const u32x4 lds_u32x4;
__device__ inline bf16x8 frag3(const lds_t* plane, int row, int lq) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<lds_u32x4*>(plane + row * ROWB + 16 * swz(row, lq)));
}

// One chunk (16 FP32 contraction elements, 64-byte rows) of this wave's TA x TB
// block of 16 x 16 tiles on v_mfma_f32_16x16x4f32. Lane (lr, lq) reads piece
// lq of its row (elements 4 lq .. 4 lq + 3) from A (at la) and from B (at lb),
// both k-contiguous; the MFMA of step e pairs element e of both, so the four
// steps together contract all 16 elements (the order of the sum over a chunk
// is a permutation of k, the same for A and B).
template <int TA, int TB>
__device__ inline void mma_f32(f4 (&acc)[TA][TB], const unsigned char* la, const unsigned char* lb, int arow,
                               int brow, int lane) {
  const int lr = lane & 15, lq = lane >> 4;
  f4 a[TA], b[TB];
#pragma unroll
  for (int i = 0; i < TA; ++i) a[i] = __builtin_bit_cast(f4, lds16(la + (arow + 16 * i + lr) * ROWB + 16 * swz(arow + 16 * i + lr, lq)));
#pragma unroll
  for (int j = 0; j < TB; ++j) b[j] = __builtin_bit_cast(f4, lds16(lb + (brow + 16 * j + lr) * ROWB + 16 * swz(brow + 16 * j + lr, lq)));
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int j = 0; j < TB; ++j)
#pragma unroll
      for (int i = 0; i < TA; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][e], b[j][e], acc[i][j], 0, 0, 0);
}

// Direct global->LDS loads and their waits, written as inline asm so that the
// compiler's wait-count pass does not track them: it cannot tell the three
// ring buffers apart across the loop and would add a conservative vmcnt(0)
// before the LDS reads of some steps. A kernel using them therefore waits for
// its own loads explicitly (every LDS read of a buffer follows a vmcnt wait
// covering that buffer's loads and a barrier). Lane l of a load writes LDS
// bytes [m0 + BYTES l, m0 + BYTES (l + 1)). No VGPR is written by these loads.
// M0 is reserved by the compiler, but the kernels using these helpers use it
// nowhere else (no indirect register indexing, message or GWS instruction),
// so clobbering it here is safe; the warning about it is silenced for these two.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ inline void dma16(const unsigned char* src, lds_t* dst) {
  const unsigned m = __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)dst);
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(m) : "memory", "m0");
}
__device__ inline void dma4(const unsigned char* src, lds_t* dst) {
  const unsigned m = __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)dst);
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off" ::"v"(src), "s"(m) : "memory", "m0");
}
// The same load with a wave-uniform 64-bit base in SGPRs and a per-lane 32-bit
// byte offset: the address arithmetic of a load is then scalar. m is the LDS
// byte address the wave's lane 0 writes (wave-uniform).
__device__ inline void dma16s(const unsigned char* base, unsigned voff, unsigned m) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(voff), "s"(base), "s"(m)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// s_waitcnt vmcnt(W) followed by s_barrier, one opaque statement: it is also a
// compiler-level memory barrier, so no LDS access moves across it
template <int W> __device__ inline void wait_vm_barrier() {
  static_assert(W >= 0 && W < 64, "vmcnt is 6 bits");
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(W) : "memory");
}

// s_waitcnt lgkmcnt(0) followed by s_barrier: every LDS read of every wave
// has returned, so the buffers they read may be refilled after it
__device__ inline void lgkm_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Loader of bf3_stream for operands whose chunks are a fixed stride apart:
// loads q < QA move A rows (chunks astride bytes apart), the others B rows
template <int NQ, int QA> struct StrideLoader {
  const unsigned char* qb[NQ];   // load q's first row in chunk 0
  long astride, bstride;
  __device__ const unsigned char* src(int q, int ch) const { return qb[q] + (long)ch * (q < QA ? astride : bstride); }
};

// The split-BF16x3 chunk loop of a TA x TB wave tile with the fragments in
// registers. Operands are chunk-major planes as above, one LDS stage holding
// A hi (REGA bytes), A lo, B hi (REGB bytes), B lo; a wave moves NQ 1 KB
// loads per chunk: load q is instruction t = NQ-major (q * 4 + wave) of the
// stage, 16 rows whose global base for chunk ch is ld.src(q, ch) (wave-uniform)
// and whose lane l reads row l / 4, swizzled piece, i.e. the per-lane offset
// voff below (the swizzle of row 16 j + l / 4 does not depend on j).
//
// Chunk c's fragments live in registers; each register is refilled from
// chunk c + 1 right after its last MFMA of chunk c, so the reads overlap the
// MFMAs without a second register set. Row tile by row tile: products hi*hi
// (p0), lo*hi (p2), hi*lo (p1) over the TB column tiles (an accumulator's
// MFMAs at least TB apart); A lo refilled after p2, A hi after p1. The B
// fragments serve every tile: the last KD tiles defer their p1, so that the
// B hi fragments are refilled after the last p2 with KD * TB MFMAs to go and
// each B lo one after its last MFMA. After p2 of tile 0 every wave has
// consumed chunk c's fragments: a barrier there (this wave's reads returned)
// frees chunk c's buffer for the loads of chunk c + 3, spread evenly over the
// MFMAs that follow. The step ends once chunk c + 2 has landed. Every read and
// load sits between two MFMAs, so the matrix pipe always has queued work
// while the wave issues them; scheduling barriers keep the order. Past the
// last chunk the loads fetch chunk 0 again into the buffer being refilled
// (free, and never read as data), so every step keeps the same wait count.
//
// With CB (compact B) the B operand is the real form of a complex matrix,
// rows 2m + part, contraction 2k + p: row (m, 0) = [Re a, -Im a], row (m, 1)
// = [Im a, Re a] over k (a = a_mk). Only rows m = [Re a, Im a] are stored
// (REGB holds half as many rows); lane lr reads row (brow + 16 j + lr) / 2
// and forms its real-form row in registers, exactly: part 0 flips the sign
// of the odd elements, part 1 swaps each pair.
//
// On return every load has landed; the caller's epilogue may reuse the LDS
// after a __syncthreads().
template <int TA, int TB, int REGA, int REGB, int NQ, bool CB = false, class Loader>
__device__ __forceinline__ void bf3_stream(f4 (&acc)[TA][TB], const lds_t* L0, const lds_t* L1, const lds_t* L2,
                                           int nc, int arow, int brow, int lane, int wave, const Loader& ld) {
  constexpr int NW = 4;
  constexpr int KD = TA > 3 ? 3 : TA > 2 ? 2 : 1;
  // MFMAs after the barrier outside the deferred tail: the slots of the loads
  constexpr int SPAN = 3 * TA * TB - 2 * TB - KD * TB;
  static_assert(SPAN >= NQ, "tile too small for the chunk loop");
  // the loads spread evenly over those slots: issued in a burst they queue up
  // in the CU's vector memory path (1 KB each) and stall the wave's MFMAs
  constexpr int LSTRIDE = SPAN / NQ;
  const int lr = lane & 15, lq = lane >> 4;
  const unsigned voff = (unsigned)((lane >> 2) * ROWB + 16 * swz(lane >> 2, lane & 3));
  auto addr = [](const lds_t* p) { return (unsigned)(uintptr_t)p; };
  const unsigned lds0 = addr(L0) + wave * 1024, lds1 = addr(L1) + wave * 1024, lds2 = addr(L2) + wave * 1024;
  auto load = [&](int q, int chunk, unsigned mbuf) {
    dma16s(ld.src(q, chunk < nc ? chunk : 0), voff, mbuf + q * NW * 1024);
  };
  // B fragment j of the plane at p (real-form row brow + 16 j + lr)
  const unsigned rot = CB && (lr & 1) ? 16u : 0u, flip = CB && !(lr & 1) ? 0x80000000u : 0u;
  auto fragb = [&](const lds_t* p, int j) -> bf16x8 {
    if constexpr (!CB) {
      return frag3(p, brow + 16 * j + lr, lq);
    } else {
      u32x4 d = __builtin_bit_cast(u32x4, frag3(p, (brow + 16 * j + lr) >> 1, lq));
#pragma unroll
      for (int e = 0; e < 4; ++e) d[e] = __builtin_amdgcn_alignbit(d[e], d[e], rot) ^ flip;
      return __builtin_bit_cast(bf16x8, d);
    }
  };
  bf16x8 ah[TA], al[TA], bh[TB], bl[TB];
#pragma unroll
  for (int q = 0; q < NQ; ++q) load(q, 0, lds0);
#pragma unroll
  for (int q = 0; q < NQ; ++q) load(q, 1, lds1);
#pragma unroll
  for (int q = 0; q < NQ; ++q) load(q, 2, lds2);
  wait_vm_barrier<2 * NQ>();                      // chunk 0 has landed
#pragma unroll
  for (int i = 0; i < TA; ++i) {
    ah[i] = frag3(L0, arow + 16 * i + lr, lq);
    al[i] = frag3(L0 + REGA, arow + 16 * i + lr, lq);
  }
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    bh[j] = fragb(L0 + 2 * REGA, j);
    bl[j] = fragb(L0 + 2 * REGA + REGB, j);
  }
  wait_vm_barrier<NQ>();                          // chunk 1 has landed
  // b0: chunk c (in registers), b1: chunk c + 1 (landed), b2: chunk c + 2
  unsigned m0b = lds0, m1b = lds1, m2b = lds2;
#define AFQ_RING_MFMA(X, Y, i, j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(X, Y, acc[i][j], 0, 0, 0)
#define AFQ_RING_SB __builtin_amdgcn_sched_barrier(0)
  for (int c = 0; c < nc; ++c) {
    const lds_t* const b1 = (const lds_t*)(uintptr_t)(m1b - wave * 1024);
    int s = 0;                                    // MFMA slot after the barrier (folds to a constant)
    // load q of chunk c + 3 after slot q * LSTRIDE
#define AFQ_RING_LOADS                                  \
  do {                                                  \
    if (s % LSTRIDE == 0 && s / LSTRIDE < NQ) {         \
      load(s / LSTRIDE, c + 3, m0b);                    \
      AFQ_RING_SB;                                      \
    }                                                   \
    ++s;                                                \
  } while (0)
#pragma unroll
    for (int i = 0; i < TA; ++i) {
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        AFQ_RING_MFMA(ah[i], bh[j], i, j);
        AFQ_RING_SB;
        if (i > 0) AFQ_RING_LOADS;
      }
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        AFQ_RING_MFMA(al[i], bh[j], i, j);
        AFQ_RING_SB;
        if (i > 0) AFQ_RING_LOADS;
      }
      if (i == 0) {
        lgkm_barrier();
        AFQ_RING_SB;
      }
      al[i] = frag3(b1 + REGA, arow + 16 * i + lr, lq);
      AFQ_RING_SB;
      if (i < TA - KD) {
#pragma unroll
        for (int j = 0; j < TB; ++j) {
          AFQ_RING_MFMA(ah[i], bl[j], i, j);
          AFQ_RING_SB;
          AFQ_RING_LOADS;
        }
        ah[i] = frag3(b1, arow + 16 * i + lr, lq);
        AFQ_RING_SB;
      }
    }
#pragma unroll
    for (int d = 0; d < KD; ++d) {
      const int i = TA - KD + d;
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        AFQ_RING_MFMA(ah[i], bl[j], i, j);
        AFQ_RING_SB;
        if (d == 0) bh[j] = fragb(b1 + 2 * REGA, j);
        if (d == KD - 1) bl[j] = fragb(b1 + 2 * REGA + REGB, j);
        AFQ_RING_SB;
      }
      ah[i] = frag3(b1, arow + 16 * i + lr, lq);
      AFQ_RING_SB;
    }
    wait_vm_barrier<NQ>();
    const unsigned t_ = m0b;
    m0b = m1b;
    m1b = m2b;
    m2b = t_;
  }
#undef AFQ_RING_LOADS
#undef AFQ_RING_SB
#undef AFQ_RING_MFMA
  wait_vm_barrier<0>();
}

}  // namespace ring
