// Internal declarations of the fixed-lineshape batched path.
#pragma once

#include "pwa_internal.h"

namespace pwa {

constexpr int kSlices = 4;         // fixed-point slices per operand (sliced FP16 format)

struct BatchArgs {
  const void* A[kSlices];  // N_D x KP amplitude operands (row-major), one plane per slice
  const void* C[kSlices];  // coupling operands: KP x 2B (row-major) per part, or
                           // [2][B][KP] per slice for the sliced format
  int KP;
  int B;
  int64_t n;               // N_D
  double* part;            // row-block partials: (hi, lo) per start
  double* part2;           // chunk partials of the row-block partials: (hi, lo) per start
  const unsigned long long* esum;   // sliced format: sum over events of the row exponents
};

constexpr int kBatchChunks = 32;   // chunks of the first stage of the per-start sum

int batched_kp(int fmt, int K);
int batched_elem_bytes(int fmt);
int batched_a_planes(int fmt);
int batched_c_planes(int fmt);
hipError_t launch_freeze(int fmt, const double* planes, int64_t stride, int64_t n,
                         const double* tbl, const int* itbl, int K, int KP, int gen,
                         void* const* out, unsigned long long* esum, hipStream_t st);
// xtx: scratch of 48 x 48 doubles (the summed X^T X)
hipError_t launch_gram(const double* planes, int64_t stride, int64_t base, int64_t n,
                       const double* tbl, const int* itbl, int K, int gen, int nblocks, double* part,
                       double* xtx, double* gram, hipStream_t st);
// sliced FP16 format (pwa_sliced.hip)
hipError_t launch_freeze_slices(const double* planes, int64_t stride, int64_t n, const double* tbl,
                                const int* itbl, int K, int KP, int gen, _Float16* q,
                                unsigned long long* esum, hipStream_t st);
hipError_t launch_sliced(const BatchArgs& a, int row_blocks, const double* C, int K, hipStream_t st);
hipError_t launch_batched(int fmt, const BatchArgs& a, int row_blocks, const double* C,
                          const double* gram, int K, double nd, double nm, double* nll,
                          hipStream_t st);

}  // namespace pwa
