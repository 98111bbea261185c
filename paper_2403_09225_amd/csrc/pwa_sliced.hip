// Sliced FP16 format of the fixed-lineshape batched path: amplitudes and
// couplings as fixed-point integer slices on the FP16 matrix cores.
//
// Why slices.  A rounding of a coupling shifts every event's log the same
// way, so the couplings need about 36 bits; the FP16 matrix cores align the
// products of one instruction to the largest and drop the low bits, so a
// floating split (hi + lo parts) loses its low parts inside the sum and
// biases it.  Products of integers below 2^18 summed below 2^24 are exact
// whatever the alignment, so each operand is cut into integer slices of 9
// bits on a common power-of-two grid (per event for the amplitudes, per
// start for the couplings; see slice4) and only integer dot products are
// formed.  Z = A c is recovered from the slice products of levels i + j <= 3
// (ten products), accurate to 2^-28 of the row's largest amplitude.
//
// This file is compiled with MFMA results in ordinary VGPRs (the epilogue
// reads every accumulator; accumulation registers would cost one move per
// value).

#include <math.h>

#include "pwa_batched.h"
#include "pwa_batched_dev.h"

namespace pwa {

// Per event: the amplitude row's exponent E_i, its four slice rows, and the
// block's sum of E_i added to *esum (integer atomics: order independent).
__global__ __launch_bounds__(256) void freeze_slices_kernel(const double* __restrict__ planes,
                                                            int64_t stride, int64_t n,
                                                            const double* __restrict__ tbl,
                                                            const int* __restrict__ itbl, int K,
                                                            int KP, int gen, _Float16* __restrict__ q,
                                                            unsigned long long* __restrict__ esum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t plane = n * KP;   // slice planes are contiguous, n x KP each
  long long e_row = 0;
  if (i < n) {
    double m = 0.0;
    for (int k = 0; k < K; ++k) {
      double re, im;
      frozen_amp(planes, stride, i, tbl, itbl, k, gen, re, im);
      m = fmax(m, fmax(fabs(re), fabs(im)));
    }
    const int E = max_exponent(m);
    e_row = E;
    const double sc = ldexp(1.0, 9 - E);
    for (int k = 0; k < K; ++k) {   // recomputed: cheaper than holding 2K values per thread
      double re, im;
      frozen_amp(planes, stride, i, tbl, itbl, k, gen, re, im);
      slice4(re * sc, q + i * KP + k, plane);
      slice4(im * sc, q + i * KP + K + k, plane);
    }
    for (int c = 2 * K; c < KP; ++c) slice4(0.0, q + i * KP + c, plane);
  }
  for (int off = 32; off > 0; off >>= 1) e_row += __shfl_xor(e_row, off);
  __shared__ long long wsum[4];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = e_row;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicAdd(esum, (unsigned long long)(wsum[0] + wsum[1] + wsum[2] + wsum[3]));
}

// Sliced coupling operands, [slice][part][b][KP] (part 0: the real column
// [Cr; -Ci] of start b, part 1: the imaginary column [Ci; Cr]), each start
// scaled by 2^(9 - G_b).  One thread per (part, b, row).
__global__ void coupling_slices_kernel(const double* __restrict__ C, int K, int KP, int B,
                                       _Float16* __restrict__ q) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * B * KP) return;
  const int part = idx / (B * KP), b = (idx / KP) % B, row = idx % KP;
  double v = 0.0;
  if (row < 2 * K) {
    const int k = row < K ? row : row - K;
    const double cr = C[2 * (b * K + k)], ci = C[2 * (b * K + k) + 1];
    v = row < K ? (part ? ci : cr) : (part ? cr : -ci);
  }
  slice4(v * ldexp(1.0, 9 - coupling_exponent(C, K, b)), q + idx, (int64_t)2 * B * KP);
}

// ------------------------------------------------------------------------
// Data term.  Per 16 x 16 tile of (events, starts), the real and imaginary
// tiles of four levels are accumulated on the FP16 matrix cores (16x16x32
// steps, one 16x16x16 step for a 16-wide tail):
//   L0 = q0.c0,  L1 = q0.c1 + q1.c0,  L2 = q0.c2 + q1.c1 + q2.c0,
//   L3 = q0.c3 + q1.c2 + q2.c1 + q3.c0.
// Every product is an integer; L0 .. L2 stay below 2^24 (at most 48 terms
// of 2^18, 2^17 + 2^17, 2^17 + 2^16 + 2^17) and are exact in FP32, L3 may
// reach 1.2 x 2^24 (one rounding, 2^-51 of the scale of Z).  Then
//   Z 2^(18 - E_i - G_b) = L0 + 2^-9 (L1 + 2^-9 (L2 + 2^-9 L3)),
// the bracket in FP32 (one rounding, 2^-33 of that scale), the sum in FP64.
// The logs: each lane keeps, per start, the running FP64 product of its
// events' |Z|^2 as a mantissa in [1/2, 1) and an integer exponent (4 events
// per step: at most 2^196 before renormalising) and takes one logarithm at
// the end; the product's rounding, 2^-53 per factor, is far below the
// format's.  An exactly zero Z, which only vanishing couplings or
// amplitudes give, is not supported.
//
// Packed tail.  When at most 8 of the tail's 16 columns are real (2K - 32
// N32 <= 8, e.g. K = 20), the tail step's upper k-groups carry the next
// slice instead of zeros, so one 16x16x16 MFMA forms two slice products:
// the tail of coupling slice s is staged as [c_s | c_(s-1)] (rows of the
// real columns; zeros under c_0) and the amplitude tails as [q0 | q1] and
// [q2 | q3] (and [q0 | 0], [q2 | 0]); then
//   L0 += [q0|0].c0, L1 += [q0|q1].[c1|c0], L2 += [q0|q1].[c2|c1] + [q2|0].c0,
//   L3 += [q0|q1].[c3|c2] + [q2|q3].[c1|c0]:
// six tail MFMAs per part instead of ten.
//
// MFMA layouts (checked on gfx950): A lane l = row l % 16, k-group l / 16;
// B lane l = k-group l / 16, column l % 16; result lane l = column l % 16,
// rows 4 (l / 16) + r.  The chunk's coupling slices sit in LDS in operand
// order: for tile t, slice s and part p, the B operand of each k-step is
// stored lane by lane (8 halves per lane for a 16x16x32 step, 4 for the
// tail), so every operand read of a wave is one contiguous block, free of
// bank conflicts.
//
// Grid: row_blocks x chunks blocks in one dimension.  Workgroups are dealt
// to the 8 XCDs in turn, so the chunk blocks of one row block are placed 8
// apart: they run on one XCD at nearly the same time and the amplitude rows
// read from HBM by the first are served to the others from that XCD's L2.
// ------------------------------------------------------------------------
constexpr int kSlicedCHB = 64;

__device__ __forceinline__ f4_t mma_h(h8_t a, h8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mma_h(h4_t a, h4_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// The ten slice products of one k-step into L[0..7] = L0r, L0i, L1r, L1i,
// L2r, L2i, L3r, L3i; deepest level first so that consecutive updates of one
// accumulator are several instructions apart.
template <typename V>
__device__ __forceinline__ void slice_products(const V* q, const V* cr, const V* ci, f4_t* L) {
  L[6] = mma_h(q[3], cr[0], L[6]);
  L[7] = mma_h(q[3], ci[0], L[7]);
  L[4] = mma_h(q[2], cr[0], L[4]);
  L[5] = mma_h(q[2], ci[0], L[5]);
  L[6] = mma_h(q[2], cr[1], L[6]);
  L[7] = mma_h(q[2], ci[1], L[7]);
  L[2] = mma_h(q[1], cr[0], L[2]);
  L[3] = mma_h(q[1], ci[0], L[3]);
  L[4] = mma_h(q[1], cr[1], L[4]);
  L[5] = mma_h(q[1], ci[1], L[5]);
  L[6] = mma_h(q[1], cr[2], L[6]);
  L[7] = mma_h(q[1], ci[2], L[7]);
  L[0] = mma_h(q[0], cr[0], L[0]);
  L[1] = mma_h(q[0], ci[0], L[1]);
  L[2] = mma_h(q[0], cr[1], L[2]);
  L[3] = mma_h(q[0], ci[1], L[3]);
  L[4] = mma_h(q[0], cr[2], L[4]);
  L[5] = mma_h(q[0], ci[2], L[5]);
  L[6] = mma_h(q[0], cr[3], L[6]);
  L[7] = mma_h(q[0], ci[3], L[7]);
}

template <int N32, int N16, bool PACK>
__global__ __launch_bounds__(256) void sliced_kernel(BatchArgs a, int nchunk) {
  static_assert(!PACK || N16 == 1, "the packed tail needs a tail step");
  constexpr int CHB = kSlicedCHB;
  constexpr int NT = CHB / 16;
  constexpr int KP = 32 * N32 + 16 * N16;
  constexpr int TSP = 16 * KP;   // halves per (tile, slice, part) operand block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int B = a.B;
  int rb = blockIdx.x, ch = 0;
  if (nchunk > 1) {
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    ch = j % nchunk;
    rb = (j / nchunk) * 8 + xcd;
  }
  const int nrb = gridDim.x / nchunk;
  const int b0 = ch * CHB;
  extern __shared__ char smem_raw[];
  _Float16* sC = (_Float16*)smem_raw;   // [NT][kSlices * 2][TSP]
  {
    // 8-byte words (4 consecutive k of one start) from [slice][part][b][KP]
    constexpr int WPR = KP / 4;
    const _Float16* src = (const _Float16*)a.C[0];
    for (int w = threadIdx.x; w < kSlices * 2 * CHB * WPR; w += blockDim.x) {
      const int sp = w / (CHB * WPR), c = (w / WPR) % CHB, k0 = 4 * (w % WPR);   // sp = 2 slice + part
      uint2 v = {0u, 0u};
      if (b0 + c < B) v = *(const uint2*)(src + ((int64_t)sp * B + b0 + c) * KP + k0);
      const int t = c >> 4, cl = c & 15;
      _Float16* blk = sC + (t * kSlices * 2 + sp) * TSP;
      if (k0 < 32 * N32) {   // 16x16x32 step k0 / 32: lane 16 kg + col holds k = 8 kg .. 8 kg + 7
        const int kg = (k0 & 31) >> 3;
        *(uint2*)(blk + (k0 >> 5) * 512 + (kg * 16 + cl) * 8 + (k0 & 7)) = v;
      } else {               // 16x16x16 tail: lane 16 kg + col holds k = 4 kg .. 4 kg + 3
        const int kg = (k0 - 32 * N32) >> 2;
        if constexpr (PACK) {
          // [c_s | c_(s-1)]: the real rows (k-groups 0, 1) of slice s go to
          // its own block and to the upper k-groups of slice s + 1's block
          const int sl = sp >> 1;
          if (kg < 2) {
            *(uint2*)(blk + N32 * 512 + (kg * 16 + cl) * 4) = v;
            if (sl + 1 < kSlices) *(uint2*)(blk + 2 * TSP + N32 * 512 + ((kg + 2) * 16 + cl) * 4) = v;
          } else if (sl == 0) {
            *(uint2*)(blk + N32 * 512 + (kg * 16 + cl) * 4) = v;   // zero padding
          }
        } else {
          *(uint2*)(blk + N32 * 512 + (kg * 16 + cl) * 4) = v;
        }
      }
    }
  }
  __syncthreads();

  const int64_t rows_per_block = (a.n + nrb - 1) / nrb;
  const int64_t r_begin = min(a.n, (int64_t)rb * rows_per_block);
  const int64_t r_end = min(a.n, r_begin + rows_per_block);
  double pm[NT];   // running product of |Z|^2: mantissa in [1/2, 1) ...
  int pe[NT];      // ... and exponent
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    pm[t] = 1.0;
    pe[t] = 0;
  }
  const int col = lane & 15, kg = lane >> 4;
  const int64_t plane = a.n * KP;
  const _Float16* A0 = (const _Float16*)a.A[0];
  for (int64_t r0 = r_begin + 16 * wave; r0 < r_end; r0 += 64) {
    // operands of rows r0 .. r0 + 15: lane = row l % 16, k-group l / 16
    const int64_t row = min(r0 + col, a.n - 1);
    h8_t q8[N32 > 0 ? N32 : 1][kSlices];
    h4_t q4[kSlices];   // tail operands; packed: [q0|0], [q0|q1], [q2|0], [q2|q3]
#pragma unroll
    for (int s = 0; s < kSlices; ++s) {
      const _Float16* ar = A0 + s * plane + row * KP;
#pragma unroll
      for (int j = 0; j < N32; ++j) q8[j][s] = *(const h8_t*)(ar + 32 * j + 8 * kg);
      if constexpr (N16 > 0 && !PACK) q4[s] = *(const h4_t*)(ar + 32 * N32 + 4 * kg);
    }
    if constexpr (PACK) {
      const int kt = 32 * N32 + 4 * (kg & 1);   // real tail columns only
      const int up = kg >> 1;                   // upper k-groups: the next slice
      const h4_t p01 = *(const h4_t*)(A0 + (0 + up) * plane + row * KP + kt);
      const h4_t p23 = *(const h4_t*)(A0 + (2 + up) * plane + row * KP + kt);
      const h4_t z = {0, 0, 0, 0};
      q4[0] = up ? z : p01;
      q4[1] = p01;
      q4[2] = up ? z : p23;
      q4[3] = p23;
    }
    bool valid[4];
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) valid[qq] = r0 + 4 * kg + qq < r_end;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      f4_t L[8];
#pragma unroll
      for (int x = 0; x < 8; ++x) L[x] = (f4_t){0.f, 0.f, 0.f, 0.f};
      const _Float16* cb = sC + t * kSlices * 2 * TSP;
#pragma unroll
      for (int j = 0; j < N32; ++j) {
        h8_t cr[kSlices], ci[kSlices];
#pragma unroll
        for (int s = 0; s < kSlices; ++s) {
          cr[s] = *(const h8_t*)(cb + (2 * s) * TSP + j * 512 + lane * 8);
          ci[s] = *(const h8_t*)(cb + (2 * s + 1) * TSP + j * 512 + lane * 8);
        }
        slice_products(q8[j], cr, ci, L);
      }
      if constexpr (N16 > 0) {
        h4_t cr[kSlices], ci[kSlices];
#pragma unroll
        for (int s = 0; s < kSlices; ++s) {
          cr[s] = *(const h4_t*)(cb + (2 * s) * TSP + N32 * 512 + lane * 4);
          ci[s] = *(const h4_t*)(cb + (2 * s + 1) * TSP + N32 * 512 + lane * 4);
        }
        if constexpr (PACK) {
          // q4 = [q0|0], [q0|q1], [q2|0], [q2|q3]; c = c0, [c1|c0], [c2|c1], [c3|c2]
          L[6] = mma_h(q4[3], cr[1], L[6]);
          L[7] = mma_h(q4[3], ci[1], L[7]);
          L[4] = mma_h(q4[2], cr[0], L[4]);
          L[5] = mma_h(q4[2], ci[0], L[5]);
          L[2] = mma_h(q4[1], cr[1], L[2]);
          L[3] = mma_h(q4[1], ci[1], L[3]);
          L[0] = mma_h(q4[0], cr[0], L[0]);
          L[1] = mma_h(q4[0], ci[0], L[1]);
          L[6] = mma_h(q4[1], cr[3], L[6]);
          L[7] = mma_h(q4[1], ci[3], L[7]);
          L[4] = mma_h(q4[1], cr[2], L[4]);
          L[5] = mma_h(q4[1], ci[2], L[5]);
        } else {
          slice_products(q4, cr, ci, L);
        }
      }
      // epilogue: Z per event in FP64, |Z|^2 into the running product
      double prod = pm[t];
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const float Rr = fmaf(0x1p-9f, fmaf(0x1p-9f, L[6][qq], L[4][qq]), L[2][qq]);
        const float Ri = fmaf(0x1p-9f, fmaf(0x1p-9f, L[7][qq], L[5][qq]), L[3][qq]);
        const double zr = fma(0x1p-9, (double)Rr, (double)L[0][qq]);
        const double zi = fma(0x1p-9, (double)Ri, (double)L[1][qq]);
        prod *= valid[qq] ? fma(zr, zr, zi * zi) : 1.0;
      }
      int es;
      pm[t] = frexp(prod, &es);
      pe[t] += es;
      // keep the scheduler from hoisting the next tile's operand reads
      // above this epilogue (they would need a second set of registers)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __shared__ double red[4][CHB][2];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double hi = ln_small64(pm[t]) + (double)pe[t] * 6.93147180369123816490e-01;
    double lo = (double)pe[t] * 1.90821492927058770002e-10;
    for (int off = 16; off < 64; off <<= 1) {
      const double oh = __shfl_xor(hi, off), ol = __shfl_xor(lo, off);
      dd_add_b(hi, lo, oh, ol);
    }
    if (kg == 0) {
      red[wave][t * 16 + col][0] = hi;
      red[wave][t * 16 + col][1] = lo;
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < CHB; b += blockDim.x) {
    double h = red[0][b][0], l = red[0][b][1];
    for (int w = 1; w < 4; ++w) dd_add_b(h, l, red[w][b][0], red[w][b][1]);
    if (b0 + b < B) {
      a.part[((int64_t)rb * B + b0 + b) * 2] = h;
      a.part[((int64_t)rb * B + b0 + b) * 2 + 1] = l;
    }
  }
}

hipError_t launch_freeze_slices(const double* planes, int64_t stride, int64_t n, const double* tbl,
                                const int* itbl, int K, int KP, int gen, _Float16* q,
                                unsigned long long* esum, hipStream_t st) {
  hipError_t e = hipMemsetAsync(esum, 0, sizeof(unsigned long long), st);
  if (e != hipSuccess || n <= 0) return e;
  hipLaunchKernelGGL(freeze_slices_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     planes, stride, n, tbl, itbl, K, KP, gen, q, esum);
  return hipGetLastError();
}

hipError_t launch_sliced(const BatchArgs& a, int row_blocks, const double* C, int K, hipStream_t st) {
  const unsigned cg = (unsigned)((a.KP * 2 * a.B + 255) / 256);
  hipLaunchKernelGGL(coupling_slices_kernel, dim3(cg), dim3(256), 0, st, C, K, a.KP, a.B,
                     (_Float16*)a.C[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nchunk = (a.B + kSlicedCHB - 1) / kSlicedCHB;
  if (nchunk > 1 && row_blocks % 8 != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(row_blocks * nchunk));
  const size_t lds = (size_t)kSlices * 2 * kSlicedCHB * a.KP * sizeof(_Float16);
  // packed tail: at most 8 real columns in the 16-wide tail step
  const bool pack = (a.KP % 32 == 16) && (2 * K - (a.KP / 32) * 32 <= 8);
  switch (a.KP) {
    case 16:
      if (pack) hipLaunchKernelGGL((sliced_kernel<0, 1, true>), grid, dim3(256), lds, st, a, nchunk);
      else hipLaunchKernelGGL((sliced_kernel<0, 1, false>), grid, dim3(256), lds, st, a, nchunk);
      break;
    case 32: hipLaunchKernelGGL((sliced_kernel<1, 0, false>), grid, dim3(256), lds, st, a, nchunk); break;
    case 48:
      if (pack) hipLaunchKernelGGL((sliced_kernel<1, 1, true>), grid, dim3(256), lds, st, a, nchunk);
      else hipLaunchKernelGGL((sliced_kernel<1, 1, false>), grid, dim3(256), lds, st, a, nchunk);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pwa
