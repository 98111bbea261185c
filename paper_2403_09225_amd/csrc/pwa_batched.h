// Internal declarations of the fixed-lineshape batched path.
#pragma once

#include "pwa_internal.h"

namespace pwa {

struct BatchArgs {
  const void* A_hi;   // N_D x KP amplitude operands (row-major)
  const void* A_lo;   // low parts (split format) or null
  const void* C_hi;   // KP x 2B coupling operands (row-major)
  const void* C_lo;   // second coupling part (FP32 and split formats) or null
  const void* C_lo2;  // third coupling part (split format) or null
  int KP;
  int B;
  int64_t n;          // N_D
  double* part;       // row-block partials: (hi, lo) per start
  double* part2;      // chunk partials of the row-block partials: (hi, lo) per start
};

constexpr int kBatchChunks = 32;   // chunks of the first stage of the per-start sum

int batched_kp(int fmt, int K);
int batched_elem_bytes(int fmt);
hipError_t launch_freeze(int fmt, const double* planes, int64_t stride, int64_t n,
                         const double* tbl, const int* itbl, int K, int KP, int gen, void* out_hi,
                         void* out_lo, hipStream_t st);
hipError_t launch_gram(const double* planes, int64_t stride, int64_t base, int64_t n,
                       const double* tbl, const int* itbl, int K, int gen, int nblocks, double* part,
                       double* gram, hipStream_t st);
hipError_t launch_batched(int fmt, const BatchArgs& a, int row_blocks, const double* C,
                          const double* gram, int K, double nd, double nm, double* nll,
                          hipStream_t st);

}  // namespace pwa
