// Launcher of the one-wave-per-SIMD exchange kernel (exchange_big.hip).
#pragma once
#include "common.h"

struct ExchBigArgs {
  const void* a[2];      // packed A planes (hi, lo) of this spin: rows n*N + a, kp columns
  const void* b[2];      // packed B planes of this spin: rows w*2N + part*N + b
  int n, kp, X, nw, spin;
  int rows;              // rows loaded per operand region and plane (set by the launcher)
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
