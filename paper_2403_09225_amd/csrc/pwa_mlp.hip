// Learned start-point proposal on the GPU: binned Dalitz histograms and the
// MLP (forward, backward, Adam) in bfloat16 on the matrix cores with FP32
// accumulation and FP32 master weights.  C ABI in include/pwa_mlp.h.
//
// Every product is one "NT" GEMM, C[m][n] = sum_k A[m][k] B[n][k], with both
// operands k-contiguous; the forward and backward passes keep each operand
// in the layout its consumer wants (activations and signals are written in
// row and in column layout by the producing epilogue), so no product reads
// a strided operand.  The epilogues fuse bias, GELU, GELU' and the bf16
// rounding.  Bias gradients and the loss are fixed-order sums.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "pwa.h"
#include "pwa_mlp.h"

namespace pwa_mlp {

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int NB = 32;   // histogram bins per axis

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU(x) = x Phi(x) and its derivative Phi(x) + x phi(x)
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_prime(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ------------------------------------------------------------------------
// Histograms.
// ------------------------------------------------------------------------
__global__ void zero_u32_kernel(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ __launch_bounds__(256) void hist_kernel(const double* __restrict__ s12,
                                                   const double* __restrict__ s13,
                                                   const int64_t* __restrict__ off, double a0,
                                                   double a1, double b0, double b1,
                                                   uint32_t* __restrict__ counts) {
  __shared__ uint32_t h[NB * NB];
  for (int i = threadIdx.x; i < NB * NB; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const int set = blockIdx.y;
  const int64_t lo = off[set], hi = off[set + 1];
  const int64_t per = (hi - lo + gridDim.x - 1) / gridDim.x;
  const int64_t e0 = lo + (int64_t)blockIdx.x * per;
  const int64_t e1 = min(hi, e0 + per);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const double x = (s12[e] - a0) / (a1 - a0) * (double)NB;
    const double y = (s13[e] - b0) / (b1 - b0) * (double)NB;
    const int i = x < 0.0 ? 0 : (x >= NB - 1 ? NB - 1 : (int)x);
    const int j = y < 0.0 ? 0 : (y >= NB - 1 ? NB - 1 : (int)y);
    atomicAdd(&h[i * NB + j], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB * NB; i += blockDim.x)
    if (h[i]) atomicAdd(&counts[(int64_t)set * NB * NB + i], h[i]);
}

// In place: the count buffer is the output buffer viewed as uint32.
__global__ void hist_norm_kernel(uint32_t* __restrict__ buf, const int64_t* __restrict__ off,
                                 int n_sets) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_sets * NB * NB) return;
  const int set = (int)(i / (NB * NB));
  const int64_t n = off[set + 1] - off[set];
  const uint32_t c = buf[i];
  ((float*)buf)[i] = n > 0 ? (float)c / (float)n : 0.0f;
}

// ------------------------------------------------------------------------
// NT GEMM on the matrix cores (bf16 x bf16 -> FP32), 64 x 64 block tile,
// each of the 4 waves a 32 x 32 quarter of 2 x 2 MFMA 16x16x16 tiles.
// Lane layout (gfx950): A lane l = row l%16 with k = 4 (l/16) .. +3; B the
// same with column l%16; result lane l = column l%16, rows 4 (l/16) + q.
// Requires K % 16 == 0 and lda, ldb multiples of 4; rows beyond M (N) are
// read clamped and never stored.
// ------------------------------------------------------------------------
enum Mode { FWD_HID = 0, FWD_OUT = 1, BWD_HID = 2, GRAD = 3 };

struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  int M, N, K, lda, ldb;
  const float* bias;   // FWD_HID, FWD_OUT
  const float* z;      // BWD_HID: pre-activations [M][ldz]
  int ldz;
  float* outf;         // FWD_HID: pre-activations; FWD_OUT: y; GRAD: gradient
  int ldo;
  uint16_t* outb;      // FWD_HID, BWD_HID: bf16 result [M][ldo]
  uint16_t* outbT;     // and its transpose [N][ldt]
  int ldt;
  int m_valid;         // FWD_OUT: rows stored
};

// gfx950's 16x16x32 bf16 MFMA over the inner dimension (A and B lanes: row
// or column l % 16, 8 consecutive k at 8 (l / 16)), one 16x16x16 step for a
// 16-wide tail (K is padded to a multiple of 16).
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

template <int MODE>
__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int r = lane & 15, kg = lane >> 4;
  const uint16_t* pa[2];
  const uint16_t* pb[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    pa[i] = g.A + (int64_t)min(m0 + 16 * i + r, g.M - 1) * g.lda;
    pb[i] = g.B + (int64_t)min(n0 + 16 * i + r, g.N - 1) * g.ldb;
  }
  f4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f4_t){0.f, 0.f, 0.f, 0.f};
  int k = 0;
  for (; k + 32 <= g.K; k += 32) {
    bf8_t a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      __builtin_memcpy(&a[i], pa[i] + k + 8 * kg, sizeof(bf8_t));
      __builtin_memcpy(&b[i], pb[i] + k + 8 * kg, sizeof(bf8_t));
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  if (k < g.K) {
    s4_t a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *(const s4_t*)(pa[i] + k + 4 * kg);
      b[i] = *(const s4_t*)(pb[i] + k + 4 * kg);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 16 * i + 4 * kg + q;
        const int n = n0 + 16 * j + r;
        if (m >= g.M || n >= g.N) continue;
        const float v = acc[i][j][q];
        if constexpr (MODE == FWD_HID) {
          const float pre = v + g.bias[n];
          g.outf[(int64_t)m * g.ldo + n] = pre;
          const uint16_t h = to_bf16(gelu(pre));
          g.outb[(int64_t)m * g.ldo + n] = h;
          g.outbT[(int64_t)n * g.ldt + m] = h;
        } else if constexpr (MODE == FWD_OUT) {
          if (m < g.m_valid) g.outf[(int64_t)m * g.ldo + n] = v + g.bias[n];
        } else if constexpr (MODE == BWD_HID) {
          const uint16_t d = to_bf16(v * gelu_prime(g.z[(int64_t)m * g.ldz + n]));
          g.outb[(int64_t)m * g.ldo + n] = d;
          g.outbT[(int64_t)n * g.ldt + m] = d;
        } else {
          g.outf[(int64_t)m * g.ldo + n] = v;
        }
      }
}

// Inputs rounded to bf16 in row and column layout; rows b >= B are zero.
__global__ void cast_input_kernel(const float* __restrict__ x, int B, int Bp, int n_in,
                                  uint16_t* __restrict__ xb, uint16_t* __restrict__ xbT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)Bp * n_in) return;
  const int b = (int)(i / n_in), c = (int)(i % n_in);
  const uint16_t h = b < B ? to_bf16(x[(int64_t)b * n_in + c]) : (uint16_t)0;
  xb[i] = h;
  xbT[(int64_t)c * Bp + b] = h;
}

// Loss and its output signal dy = 2 (y - t) / (B n_out), rounded to bf16,
// in row and column layout (zero outside the true batch and outputs).  One
// block; the loss is a fixed-order FP64 sum.
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ y,
                                                   const float* __restrict__ t, int B, int Bp,
                                                   int n_out, int Op, uint16_t* __restrict__ dy,
                                                   uint16_t* __restrict__ dyT,
                                                   double* __restrict__ loss) {
  __shared__ double part[256];
  double s = 0.0;
  const float scale = 2.0f / ((float)B * (float)n_out);
  for (int i = threadIdx.x; i < Bp * Op; i += blockDim.x) {
    const int b = i / Op, o = i % Op;
    float d = 0.0f;
    if (b < B && o < n_out) d = y[b * n_out + o] - t[b * n_out + o];
    s += (double)d * (double)d;
    const uint16_t h = to_bf16(scale * d);
    dy[i] = h;
    dyT[(int64_t)o * Bp + b] = h;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0] / ((double)B * (double)n_out);
}

// Bias gradient: row sums of a column-layout signal [rows][Bp], in order.
__global__ void bias_grad_kernel(const uint16_t* __restrict__ sT, int rows, int Bp,
                                 float* __restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= rows) return;
  float s = 0.0f;
  for (int b = 0; b < Bp; ++b) s += from_bf16(sT[(int64_t)o * Bp + b]);
  out[o] = s;
}

__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, float wd, float c1, float c2, uint16_t* __restrict__ wbf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * w[i]);
  w[i] = wi;
  wbf[i] = to_bf16(wi);
}

__global__ void cast_packed_kernel(const float* __restrict__ w, int64_t n, uint16_t* __restrict__ wbf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wbf[i] = to_bf16(w[i]);
}

// Transposed bf16 copy of a row-major W [rows][cols] into WT [cols][ldt]
// (columns rows .. ldt-1 zero).
__global__ void cast_transposed_kernel(const float* __restrict__ W, int rows, int cols, int ldt,
                                       uint16_t* __restrict__ WT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)cols * ldt) return;
  const int c = (int)(i / ldt), r = (int)(i % ldt);
  WT[i] = r < rows ? to_bf16(W[(int64_t)r * cols + c]) : (uint16_t)0;
}

// ------------------------------------------------------------------------
// Host side.
// ------------------------------------------------------------------------
inline int up16(int x) { return (x + 15) / 16 * 16; }
inline size_t up256(size_t x) { return (x + 255) / 256 * 256; }

bool dims_ok(const pwa_mlp_dims* d) {
  return d && d->n_in > 0 && d->n_h1 > 0 && d->n_h2 > 0 && d->n_out > 0 && d->n_in % 16 == 0 &&
         d->n_h1 % 16 == 0 && d->n_h2 % 16 == 0 && d->n_in <= 65536 && d->n_h1 <= 65536 &&
         d->n_h2 <= 65536 && d->n_out <= 65536;
}

struct Offsets {
  size_t W1, b1, W2, b2, W3, b3, n;
};
Offsets param_offsets(const pwa_mlp_dims* d) {
  Offsets o;
  o.W1 = 0;
  o.b1 = o.W1 + (size_t)d->n_h1 * d->n_in;
  o.W2 = o.b1 + d->n_h1;
  o.b2 = o.W2 + (size_t)d->n_h2 * d->n_h1;
  o.W3 = o.b2 + d->n_h2;
  o.b3 = o.W3 + (size_t)d->n_out * d->n_h2;
  o.n = o.b3 + d->n_out;
  return o;
}

struct WsLayout {
  size_t xb, xbT, z1, h1, h1T, z2, h2, h2T, dy, dyT, dz2, dz2T, dz1, dz1T, total;
  int Bp, Op;
};
WsLayout ws_layout(const pwa_mlp_dims* d, int batch) {
  WsLayout L;
  L.Bp = up16(batch);
  L.Op = up16(d->n_out);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = up256(off + bytes);
    return o;
  };
  const size_t B = L.Bp;
  L.xb = take(2 * B * d->n_in);
  L.xbT = take(2 * B * d->n_in);
  L.z1 = take(4 * B * d->n_h1);
  L.h1 = take(2 * B * d->n_h1);
  L.h1T = take(2 * B * d->n_h1);
  L.z2 = take(4 * B * d->n_h2);
  L.h2 = take(2 * B * d->n_h2);
  L.h2T = take(2 * B * d->n_h2);
  L.dy = take(2 * B * L.Op);
  L.dyT = take(2 * B * L.Op);
  L.dz2 = take(2 * B * d->n_h2);
  L.dz2T = take(2 * B * d->n_h2);
  L.dz1 = take(2 * B * d->n_h1);
  L.dz1T = take(2 * B * d->n_h1);
  L.total = off;
  return L;
}

template <int MODE>
hipError_t gemm(const GemmArgs& g, hipStream_t st) {
  const dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
  hipLaunchKernelGGL(gemm_nt_kernel<MODE>, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// Device scratch of pwa_mlp_forward_noalloc: a fixed array in the library's
// code object (each GPU holds its own copy for the life of the process).
// Host code never uses its name as an address: the device address is looked
// up once per device with hipGetSymbolAddress and kept here.
constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device (null on a HIP error).
char* scratch_of_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = (char*)p;
  }
  return g_scratch_ptr[dev];
}

int forward_into(const pwa_mlp_dims* d, const float* w, const uint16_t* wbf, const float* x,
                 int32_t batch, float* y, char* b, hipStream_t st);

}  // namespace pwa_mlp

using namespace pwa_mlp;

extern "C" {

int pwa_hist2d(const double* d_s12, const double* d_s13, const int64_t* d_offsets, int32_t n_sets,
               double parent_mass, const double* h_masses, float* d_out, hipStream_t st) {
  if (!d_offsets || !d_out || !h_masses || n_sets < 1 || n_sets > 65535) return PWA_E_INVALID;
  if (!d_s12 || !d_s13) return PWA_E_INVALID;
  const double m1 = h_masses[0], m2 = h_masses[1], m3 = h_masses[2];
  const double a0 = (m1 + m2) * (m1 + m2), a1 = (parent_mass - m3) * (parent_mass - m3);
  const double b0 = (m1 + m3) * (m1 + m3), b1 = (parent_mass - m2) * (parent_mass - m2);
  if (!(a1 > a0) || !(b1 > b0)) return PWA_E_INVALID;
  const int64_t nb = (int64_t)n_sets * NB * NB;
  hipLaunchKernelGGL(zero_u32_kernel, dim3(blocks(nb)), dim3(256), 0, st, (uint32_t*)d_out, nb);
  if (hipGetLastError() != hipSuccess) return PWA_E_HIP;
  hipLaunchKernelGGL(hist_kernel, dim3(8, n_sets), dim3(256), 0, st, d_s12, d_s13, d_offsets, a0,
                     a1, b0, b1, (uint32_t*)d_out);
  if (hipGetLastError() != hipSuccess) return PWA_E_HIP;
  hipLaunchKernelGGL(hist_norm_kernel, dim3(blocks(nb)), dim3(256), 0, st, (uint32_t*)d_out,
                     d_offsets, n_sets);
  return hipGetLastError() == hipSuccess ? PWA_OK : PWA_E_HIP;
}

int64_t pwa_mlp_n_params(const pwa_mlp_dims* d) {
  return dims_ok(d) ? (int64_t)param_offsets(d).n : 0;
}

int64_t pwa_mlp_n_transposed(const pwa_mlp_dims* d) {
  if (!dims_ok(d)) return 0;
  return (int64_t)d->n_h1 * d->n_h2 + (int64_t)d->n_h2 * up16(d->n_out);
}

size_t pwa_mlp_workspace_bytes(const pwa_mlp_dims* d, int32_t batch) {
  if (!dims_ok(d) || batch < 1 || batch > 65536) return 0;
  return ws_layout(d, batch).total;
}

int pwa_mlp_cast(const pwa_mlp_dims* d, const float* w, uint16_t* wbf, uint16_t* wtbf,
                 hipStream_t st) {
  if (!dims_ok(d) || !w || !wbf || !wtbf) return PWA_E_INVALID;
  const Offsets o = param_offsets(d);
  hipLaunchKernelGGL(cast_packed_kernel, dim3(blocks(o.n)), dim3(256), 0, st, w, (int64_t)o.n, wbf);
  const int Op = up16(d->n_out);
  // W2^T [n_h1][n_h2], then W3^T [n_h2][Op]
  hipLaunchKernelGGL(cast_transposed_kernel, dim3(blocks((int64_t)d->n_h1 * d->n_h2)), dim3(256), 0,
                     st, w + o.W2, d->n_h2, d->n_h1, d->n_h2, wtbf);
  hipLaunchKernelGGL(cast_transposed_kernel, dim3(blocks((int64_t)d->n_h2 * Op)), dim3(256), 0, st,
                     w + o.W3, d->n_out, d->n_h2, Op, wtbf + (size_t)d->n_h1 * d->n_h2);
  return hipGetLastError() == hipSuccess ? PWA_OK : PWA_E_HIP;
}

int pwa_mlp_forward(const pwa_mlp_dims* d, const float* w, const uint16_t* wbf, const float* x,
                    int32_t batch, float* y, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!dims_ok(d) || !w || !wbf || !x || !y || batch < 1 || batch > 65536) return PWA_E_INVALID;
  const WsLayout L = ws_layout(d, batch);
  if (!ws || ((uintptr_t)ws % 256) != 0 || ws_bytes < L.total) return PWA_E_WORKSPACE;
  return forward_into(d, w, wbf, x, batch, y, (char*)ws, st);
}

int pwa_mlp_forward_noalloc(const pwa_mlp_dims* d, const float* w, const uint16_t* wbf,
                            const float* x, int32_t batch, float* y, hipStream_t st) {
  if (!dims_ok(d) || !w || !wbf || !x || !y || batch < 1 || batch > 65536) return PWA_E_INVALID;
  // the forward pass writes the buffers in front of the first backward one
  if (ws_layout(d, batch).dy > kScratchBytes) return PWA_E_WORKSPACE;
  char* b = scratch_of_current_device();
  if (!b) return PWA_E_HIP;
  return forward_into(d, w, wbf, x, batch, y, b, st);
}

}  // extern "C"

namespace pwa_mlp {

int forward_into(const pwa_mlp_dims* d, const float* w, const uint16_t* wbf, const float* x,
                 int32_t batch, float* y, char* b, hipStream_t st) {
  const WsLayout L = ws_layout(d, batch);
  const Offsets o = param_offsets(d);
  const int Bp = L.Bp;
  uint16_t *xb = (uint16_t*)(b + L.xb), *xbT = (uint16_t*)(b + L.xbT);
  hipLaunchKernelGGL(cast_input_kernel, dim3(blocks((int64_t)Bp * d->n_in)), dim3(256), 0, st, x,
                     batch, Bp, d->n_in, xb, xbT);
  if (hipGetLastError() != hipSuccess) return PWA_E_HIP;
  GemmArgs g = {};
  // layer 1
  g.A = xb; g.lda = d->n_in; g.B = wbf + o.W1; g.ldb = d->n_in;
  g.M = Bp; g.N = d->n_h1; g.K = d->n_in; g.bias = w + o.b1;
  g.outf = (float*)(b + L.z1); g.ldo = d->n_h1;
  g.outb = (uint16_t*)(b + L.h1); g.outbT = (uint16_t*)(b + L.h1T); g.ldt = Bp;
  if (gemm<FWD_HID>(g, st) != hipSuccess) return PWA_E_HIP;
  // layer 2
  g = GemmArgs{};
  g.A = (uint16_t*)(b + L.h1); g.lda = d->n_h1; g.B = wbf + o.W2; g.ldb = d->n_h1;
  g.M = Bp; g.N = d->n_h2; g.K = d->n_h1; g.bias = w + o.b2;
  g.outf = (float*)(b + L.z2); g.ldo = d->n_h2;
  g.outb = (uint16_t*)(b + L.h2); g.outbT = (uint16_t*)(b + L.h2T); g.ldt = Bp;
  if (gemm<FWD_HID>(g, st) != hipSuccess) return PWA_E_HIP;
  // output layer
  g = GemmArgs{};
  g.A = (uint16_t*)(b + L.h2); g.lda = d->n_h2; g.B = wbf + o.W3; g.ldb = d->n_h2;
  g.M = Bp; g.N = d->n_out; g.K = d->n_h2; g.bias = w + o.b3;
  g.outf = y; g.ldo = d->n_out; g.m_valid = batch;
  if (gemm<FWD_OUT>(g, st) != hipSuccess) return PWA_E_HIP;
  return PWA_OK;
}

}  // namespace pwa_mlp

extern "C" {

int pwa_mlp_backward(const pwa_mlp_dims* d, const uint16_t* wtbf, const float* y, const float* t,
                     int32_t batch, void* ws, size_t ws_bytes, float* grad, double* loss,
                     hipStream_t st) {
  if (!dims_ok(d) || !wtbf || !y || !t || !grad || !loss || batch < 1 || batch > 65536)
    return PWA_E_INVALID;
  const WsLayout L = ws_layout(d, batch);
  if (!ws || ((uintptr_t)ws % 256) != 0 || ws_bytes < L.total) return PWA_E_WORKSPACE;
  char* b = (char*)ws;
  const Offsets o = param_offsets(d);
  const int Bp = L.Bp, Op = L.Op;
  uint16_t *dy = (uint16_t*)(b + L.dy), *dyT = (uint16_t*)(b + L.dyT);
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, st, y, t, batch, Bp, d->n_out, Op, dy, dyT,
                     loss);
  if (hipGetLastError() != hipSuccess) return PWA_E_HIP;
  const uint16_t* W2T = wtbf;
  const uint16_t* W3T = wtbf + (size_t)d->n_h1 * d->n_h2;
  GemmArgs g = {};
  // dW3 = dy^T h2, db3
  g.A = dyT; g.lda = Bp; g.B = (uint16_t*)(b + L.h2T); g.ldb = Bp;
  g.M = d->n_out; g.N = d->n_h2; g.K = Bp; g.outf = grad + o.W3; g.ldo = d->n_h2;
  if (gemm<GRAD>(g, st) != hipSuccess) return PWA_E_HIP;
  hipLaunchKernelGGL(bias_grad_kernel, dim3(blocks(d->n_out)), dim3(256), 0, st, dyT, d->n_out, Bp,
                     grad + o.b3);
  // dz2 = (dy W3) * GELU'(z2)
  g = GemmArgs{};
  g.A = dy; g.lda = Op; g.B = W3T; g.ldb = Op;
  g.M = Bp; g.N = d->n_h2; g.K = Op; g.z = (float*)(b + L.z2); g.ldz = d->n_h2;
  g.outb = (uint16_t*)(b + L.dz2); g.ldo = d->n_h2; g.outbT = (uint16_t*)(b + L.dz2T); g.ldt = Bp;
  if (gemm<BWD_HID>(g, st) != hipSuccess) return PWA_E_HIP;
  // dW2 = dz2^T h1, db2
  g = GemmArgs{};
  g.A = (uint16_t*)(b + L.dz2T); g.lda = Bp; g.B = (uint16_t*)(b + L.h1T); g.ldb = Bp;
  g.M = d->n_h2; g.N = d->n_h1; g.K = Bp; g.outf = grad + o.W2; g.ldo = d->n_h1;
  if (gemm<GRAD>(g, st) != hipSuccess) return PWA_E_HIP;
  hipLaunchKernelGGL(bias_grad_kernel, dim3(blocks(d->n_h2)), dim3(256), 0, st,
                     (uint16_t*)(b + L.dz2T), d->n_h2, Bp, grad + o.b2);
  // dz1 = (dz2 W2) * GELU'(z1)
  g = GemmArgs{};
  g.A = (uint16_t*)(b + L.dz2); g.lda = d->n_h2; g.B = W2T; g.ldb = d->n_h2;
  g.M = Bp; g.N = d->n_h1; g.K = d->n_h2; g.z = (float*)(b + L.z1); g.ldz = d->n_h1;
  g.outb = (uint16_t*)(b + L.dz1); g.ldo = d->n_h1; g.outbT = (uint16_t*)(b + L.dz1T); g.ldt = Bp;
  if (gemm<BWD_HID>(g, st) != hipSuccess) return PWA_E_HIP;
  // dW1 = dz1^T x, db1
  g = GemmArgs{};
  g.A = (uint16_t*)(b + L.dz1T); g.lda = Bp; g.B = (uint16_t*)(b + L.xbT); g.ldb = Bp;
  g.M = d->n_h1; g.N = d->n_in; g.K = Bp; g.outf = grad + o.W1; g.ldo = d->n_in;
  if (gemm<GRAD>(g, st) != hipSuccess) return PWA_E_HIP;
  hipLaunchKernelGGL(bias_grad_kernel, dim3(blocks(d->n_h1)), dim3(256), 0, st,
                     (uint16_t*)(b + L.dz1T), d->n_h1, Bp, grad + o.b1);
  return hipGetLastError() == hipSuccess ? PWA_OK : PWA_E_HIP;
}

int pwa_mlp_adam(const pwa_mlp_dims* d, float* w, float* m, float* v, const float* g, int32_t step,
                 float lr, float b1, float b2, float eps, float wd, uint16_t* wbf, uint16_t* wtbf,
                 hipStream_t st) {
  if (!dims_ok(d) || !w || !m || !v || !g || !wbf || !wtbf || step < 1) return PWA_E_INVALID;
  if (!(lr > 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps >= 0.0f) ||
      !(wd >= 0.0f))
    return PWA_E_INVALID;
  const Offsets o = param_offsets(d);
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(o.n)), dim3(256), 0, st, w, m, v, g, (int64_t)o.n,
                     lr, b1, b2, eps, wd, c1, c2, wbf);
  if (hipGetLastError() != hipSuccess) return PWA_E_HIP;
  const int Op = up16(d->n_out);
  hipLaunchKernelGGL(cast_transposed_kernel, dim3(blocks((int64_t)d->n_h1 * d->n_h2)), dim3(256), 0,
                     st, w + o.W2, d->n_h2, d->n_h1, d->n_h2, wtbf);
  hipLaunchKernelGGL(cast_transposed_kernel, dim3(blocks((int64_t)d->n_h2 * Op)), dim3(256), 0, st,
                     w + o.W3, d->n_out, d->n_h2, Op, wtbf + (size_t)d->n_h1 * d->n_h2);
  return hipGetLastError() == hipSuccess ? PWA_OK : PWA_E_HIP;
}

}  // extern "C"
