// Launcher of the one-wave-per-SIMD exchange kernel (exchange_big.hip).
#pragma once
#include "common.h"

struct ExchBigArgs {
  const void* a[2];      // packed A planes (hi, lo) of this spin: rows n*N + a, chunk-major in k
  const void* b[2];      // packed B planes of this spin: rows w*2N + part*N + b, chunk-major in k
  int n, kp, X, nw, spin;
  long rows_a, rows_b;   // rows of the packed A / B arrays (including the zero padding rows)
  int raster;            // 1: XCD-aware tile order (set by the launcher)
  double2* tro;
  double2* troo;
};

// true when the one-wave-per-SIMD kernel handles this precision and N
bool exch_big_supported(int prec, int n);
// zero rows the packed operands must carry past their last real row
inline int exch_big_pad_rows() { return 640; }
int exchange_big_launch(const ExchBigArgs& g, int prec, hipStream_t st);
// granularity of the contraction length of the packed operands
int exch_big_kchunk();
// k-chunk of the chunk-major packed layout the kernel reads
int exch_big_kchunk_major();
