// Microbenchmarks of the peaks that bound the hot path's kernels: fp32 and
// bf16 matrix-core throughput, fp32 vector FMA throughput and LDS read
// bandwidth.  Each kernel keeps every wave of a full grid busy on one kind of
// instruction with enough independent work per wave to hide its latency, and
// writes one value per thread so nothing is optimised away.  The caller times
// the launch; the work per launch is returned by tt_peak_work.
#include "common.h"

namespace ttgfx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kPeakThreads = 256;
constexpr int kChains = 8;  // independent accumulators per wave

// fp32 MFMA: v_mfma_f32_16x16x4_f32 is 2 * 16 * 16 * 4 = 2048 flop.
__global__ void __launch_bounds__(kPeakThreads) peak_mfma_f32(int iters, float *out) {
  const float a = 1.0f + 1e-7f * (float)threadIdx.x, b = 0.999f;
  v4f acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// bf16 MFMA: v_mfma_f32_16x16x32_bf16 is 2 * 16 * 16 * 32 = 16384 flop.
__global__ void __launch_bounds__(kPeakThreads) peak_mfma_bf16(int iters, float *out) {
  v8bf a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(1.0f + 0.01f * j);
    b[j] = (__bf16)(0.5f - 0.01f * j);
  }
  v4f acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// fp32 vector FMA (unpacked): 16 independent chains per lane, 2 flop each.
__global__ void __launch_bounds__(kPeakThreads) peak_valu_f32(int iters, float *out) {
  float x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = 1e-3f * (float)(threadIdx.x + c);
  const float m = 0.9999f, k = 1e-6f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 16; ++c) x[c] = __builtin_fmaf(x[c], m, k);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 16; ++c) s += x[c];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// LDS reads: every lane reads 16 bytes per instruction from a 16 KiB table at
// consecutive addresses (conflict-free), 8 reads in flight per lane.
__global__ void __launch_bounds__(kPeakThreads) peak_lds_b128(int iters, float *out) {
  __shared__ v4f tab[1024];
  for (int i = threadIdx.x; i < 1024; i += kPeakThreads) tab[i] = v4f{(float)i, 1.f, 2.f, 3.f};
  __syncthreads();
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
  int base = threadIdx.x;
  for (int i = 0; i < iters; ++i) {
    v4f r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = tab[(base + 128 * u) & 1023];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += r[u];
    base = (base + 64) & 1023;
  }
  out[blockIdx.x * kPeakThreads + threadIdx.x] = acc[0] + acc[1] + acc[2] + acc[3];
}

}  // namespace
}  // namespace ttgfx

using namespace ttgfx;

extern "C" {

// Kinds: 0 fp32 MFMA, 1 bf16 MFMA, 2 fp32 vector FMA, 3 LDS b128 reads.
// Work per launch of (blocks, iters): flop for kinds 0-2, bytes for kind 3.
double tt_peak_work(int kind, int32_t blocks, int32_t iters) {
  const double waves = (double)blocks * (kPeakThreads / 64);
  switch (kind) {
    case 0: return waves * iters * kChains * 2048.0;
    case 1: return waves * iters * kChains * 16384.0;
    case 2: return (double)blocks * kPeakThreads * iters * 16 * 2.0;
    case 3: return (double)blocks * kPeakThreads * iters * 8 * 16.0;
    default: return -1.0;
  }
}

// Launches one microbenchmark kernel on `stream`; out: (dev) float
// [blocks * 256].  Asynchronous; the caller times it (for instance with
// events on the same stream).
int tt_peak_launch(int kind, int32_t blocks, int32_t iters, float *out, void *stream) {
  if (blocks < 1 || iters < 1 || !out) return set_error(TT_ERR_ARG, "peak: blocks, iters >= 1 and out required");
  hipStream_t s = (hipStream_t)stream;
  switch (kind) {
    case 0: hipLaunchKernelGGL(peak_mfma_f32, dim3(blocks), dim3(kPeakThreads), 0, s, iters, out); break;
    case 1: hipLaunchKernelGGL(peak_mfma_bf16, dim3(blocks), dim3(kPeakThreads), 0, s, iters, out); break;
    case 2: hipLaunchKernelGGL(peak_valu_f32, dim3(blocks), dim3(kPeakThreads), 0, s, iters, out); break;
    case 3: hipLaunchKernelGGL(peak_lds_b128, dim3(blocks), dim3(kPeakThreads), 0, s, iters, out); break;
    default: return set_error(TT_ERR_ARG, "peak: unknown kind %d", kind);
  }
  return launch_check("peak microbenchmark");
}

}  // extern "C"
