// Measurement aid for the roofline figures: the throughput of the matrix
// cores when a kernel does nothing but issue independent MFMAs of one kind
// on register operands, and the shader clock they run at under that load.
// The published dense peaks assume the 2.4 GHz peak clock; under a sustained
// MFMA load the clock settles lower, and this kernel measures where.
//
// Each wave keeps four independent accumulators and issues `iters` rounds
// of four MFMAs; workgroup 0's first thread reads the shader clock counter
// (s_memtime) and the constant 100 MHz counter (s_memrealtime) at its start
// and end.
#include "common.h"
#include "kernels.h"

namespace adg {

namespace {

typedef int i32x8c __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8c __attribute__((ext_vector_type(8)));
typedef int i32x4c __attribute__((ext_vector_type(4)));

// KIND 0: FP8 e4m3 32x32x64, 1: BF16 32x32x16, 2: FP32 32x32x2.
template <int KIND>
__global__ __launch_bounds__(256) void k_mfma_ceiling(const int* __restrict__ in, float* __restrict__ out,
                                                      unsigned long long* __restrict__ clk, int iters) {
  const int t = threadIdx.x;
  i32x8c a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = in[(t * 8 + i) & 1023];
    b[i] = in[(t * 8 + i + 512) & 1023];
  }
  unsigned long long c0 = 0, r0 = 0;
  if (t == 0) {
    c0 = __builtin_amdgcn_s_memtime();
    r0 = __builtin_amdgcn_s_memrealtime();
  }
  const float fa = (float)(a[0] & 0xFFFF) * 1e-6f, fb = (float)(b[0] & 0xFFFF) * 1e-6f;
  const bf16x8c ab = __builtin_bit_cast(bf16x8c, (i32x4c){a[0], a[1], a[2], a[3]});
  const bf16x8c bb = __builtin_bit_cast(bf16x8c, (i32x4c){b[0], b[1], b[2], b[3]});
  f32x16 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = (f32x16){0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (KIND == 0) acc[q] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc[q], 0, 0, 0, 0, 0, 0);
      else if (KIND == 1) acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, bb, acc[q], 0, 0, 0);
      else acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa, fb, acc[q], 0, 0, 0);
    }
  }
  float res = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) res += acc[q][0] + acc[q][15];
  out[(size_t)blockIdx.x * 256 + t] = res;
  if (t == 0 && blockIdx.x == 0) {
    clk[0] = __builtin_amdgcn_s_memtime() - c0;
    clk[1] = __builtin_amdgcn_s_memrealtime() - r0;
  }
}

}  // namespace

int mfma_ceiling_grid() { return 1024; }

hipError_t launch_mfma_ceiling(int kind, const int* in, float* out, unsigned long long* clk, int iters,
                               hipStream_t st) {
  const unsigned G = (unsigned)mfma_ceiling_grid();
  if (kind == 0) k_mfma_ceiling<0><<<G, 256, 0, st>>>(in, out, clk, iters);
  else if (kind == 1) k_mfma_ceiling<1><<<G, 256, 0, st>>>(in, out, clk, iters);
  else if (kind == 2) k_mfma_ceiling<2><<<G, 256, 0, st>>>(in, out, clk, iters);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace adg
