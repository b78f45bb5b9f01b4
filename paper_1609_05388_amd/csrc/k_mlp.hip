// Learned form (a method extension, not in the paper): a small MLP that
// predicts log(r / d) for the target-dimension search from sketch features.
//
// Network: 67 inputs (padded to 80) -> 256 -> 256 -> 256 (ReLU) -> 1.
// Weights are BF16 copies of FP32 master weights; every product runs on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation; activations are rounded to
// BF16 as the next layer's operand.  Training minimises the pinball (quantile)
// loss at level tau of the target log(r / d) with Adam on the FP32 masters.
//
// Parameter block (FP32 masters and their BF16 copy share one layout):
//   W1 [256][80], b1 [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256],
//   w4 [256], b4 [1]   (offsets in mlp_layout()).
#include "common.h"
#include "kernels.h"

namespace adg {

// ------------------------------------------------------------------ layout
MlpLayout mlp_layout() {
  MlpLayout L;
  L.in = 67;
  L.in_pad = 80;
  L.hidden = 256;
  L.W1 = 0;
  L.b1 = L.W1 + L.hidden * L.in_pad;
  L.W2 = L.b1 + L.hidden;
  L.b2 = L.W2 + L.hidden * L.hidden;
  L.W3 = L.b2 + L.hidden;
  L.b3 = L.W3 + L.hidden * L.hidden;
  L.w4 = L.b3 + L.hidden;
  L.b4 = L.w4 + L.hidden;
  L.total = L.b4 + 4;
  return L;
}

// Operand view: element (r, k) = src[r * ld_r + k * ld_k], FP32 or BF16.
struct Opnd {
  const void* p;
  int64_t ld_r, ld_k;
  int rows, cols;     // bounds (r < rows, k < cols), zero outside
  int is_bf16;
  __device__ __bf16 get(int r, int k) const {
    if (r >= rows || k >= cols) return (__bf16)0.0f;
    const int64_t o = (int64_t)r * ld_r + (int64_t)k * ld_k;
    return is_bf16 ? static_cast<const __bf16*>(p)[o] : (__bf16) static_cast<const float*>(p)[o];
  }
};

// C[i][j] (+)= sum_k A(i, k) B(j, k) over k < K, one wave per 32 x 32 tile.
// Lane l holds A(i = l % 32, k0 + 8 (l / 32) + e) and B(j = l % 32, same k),
// e < 8 (the v_mfma_f32_32x32x16_bf16 operand layout).  Epilogue: optional
// bias[j], optional ReLU; writes FP32 C and, if Cb != NULL, a BF16 copy.
__global__ __launch_bounds__(64) void k_mlp_gemm(Opnd A, Opnd B, int M, int N, int K, const float* __restrict__ bias,
                                                 int relu, int accumulate, float* __restrict__ C, int64_t ldc,
                                                 __bf16* __restrict__ Cb, int64_t ldcb) {
  const int tiles_n = (N + 31) / 32;
  const int i0 = (blockIdx.x / tiles_n) * 32, j0 = (blockIdx.x % tiles_n) * 32;
  const int lane = threadIdx.x, li = lane & 31, lh = lane >> 5;
  f32x16 acc = (f32x16){0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + 8 * lh + e;
      a[e] = k < K ? A.get(i0 + li, k) : (__bf16)0.0f;
      b[e] = k < K ? B.get(j0 + li, k) : (__bf16)0.0f;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = i0 + (v >> 2) * 8 + lh * 4 + (v & 3), j = j0 + li;
    if (i >= M || j >= N) continue;
    float z = acc[v];
    if (accumulate) z += C[(int64_t)i * ldc + j];
    if (bias) z += bias[j];
    if (relu) z = fmaxf(z, 0.0f);
    C[(int64_t)i * ldc + j] = z;
    if (Cb) Cb[(int64_t)i * ldcb + j] = (__bf16)z;
  }
}

// out[b] = sum_h A3[b][h] * w4[h] + b4 (w4 as its BF16 value), one wave per sample.
__global__ void k_mlp_head(const float* __restrict__ A3, const __bf16* __restrict__ w4b, const float* __restrict__ b4,
                           int B, int H, float* __restrict__ out) {
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b >= B) return;
  float s = 0.0f;
  for (int h = lane; h < H; h += 64) s += A3[(int64_t)b * H + h] * (float)w4b[h];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) out[b] = s + b4[0];
}

// Pinball loss at level tau of u = y - out: L = mean(max(tau u, (tau - 1) u));
// g[b] = dL/dout_b = (u > 0 ? -tau : 1 - tau) / B.  loss[0] = L (one block).
__global__ void k_mlp_loss(const float* __restrict__ out, const float* __restrict__ y, int B, float tau,
                           float* __restrict__ g, float* __restrict__ loss) {
  __shared__ float sh[256];
  float s = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) {
    const float u = y[b] - out[b];
    s += u > 0.0f ? tau * u : (tau - 1.0f) * u;
    g[b] = (u > 0.0f ? -tau : 1.0f - tau) / (float)B;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) loss[0] = sh[0] / (float)B;
}

// Head backward: dZ3[b][h] = g[b] * w4[h] * (Z3 > 0); grad w4[h] = sum_b g[b] A3[b][h]
// (A3 = relu(Z3)), grad b4 = sum_b g[b].  One thread per hidden unit h.
__global__ void k_mlp_head_bwd(const float* __restrict__ A3, const float* __restrict__ g,
                               const __bf16* __restrict__ w4b, int B, int H, float* __restrict__ dZ3,
                               float* __restrict__ gw4, float* __restrict__ gb4) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  if (h < H) {
    float s = 0.0f;
    const float w = (float)w4b[h];
    for (int b = 0; b < B; ++b) {
      const float a = A3[(int64_t)b * H + h];
      s += g[b] * a;
      dZ3[(int64_t)b * H + h] = a > 0.0f ? g[b] * w : 0.0f;
    }
    gw4[h] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += g[b];
    gb4[0] = s;
  }
}

// dZ[b][h] *= (A[b][h] > 0): ReLU gate of the layer below (A = its activation).
__global__ void k_mlp_relu_gate(float* __restrict__ dZ, const float* __restrict__ A, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count && !(A[e] > 0.0f)) dZ[e] = 0.0f;
}

// gb[h] = sum_b dZ[b][h]
__global__ void k_mlp_bias_grad(const float* __restrict__ dZ, int B, int H, float* __restrict__ gb) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  if (h >= H) return;
  float s = 0.0f;
  for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * H + h];
  gb[h] = s;
}

// Adam on the FP32 masters (bias-corrected), then refresh the BF16 copy.
__global__ void k_mlp_adam(float* __restrict__ p, __bf16* __restrict__ pb, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, int64_t count, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  const float q = p[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[e] = q;
  pb[e] = (__bf16)q;
}

__global__ void k_to_bf16(const float* __restrict__ src, __bf16* __restrict__ dst, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) dst[e] = (__bf16)src[e];
}

// ---------------------------------------------------------------- drivers
static inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

static hipError_t gemm(Opnd A, Opnd B, int M, int N, int K, const float* bias, int relu, int acc, float* C,
                       int64_t ldc, __bf16* Cb, int64_t ldcb, hipStream_t st) {
  const int tiles = ((M + 31) / 32) * ((N + 31) / 32);
  k_mlp_gemm<<<(unsigned)tiles, 64, 0, st>>>(A, B, M, N, K, bias, relu, acc, C, ldc, Cb, ldcb);
  return hipGetLastError();
}

// Forward of a batch: X (B x in_pad, BF16 features), BF16 weights pb, FP32
// biases from p.  Saves Z/A per layer in ws (FP32 A1..A3 and BF16 copies).
hipError_t mlp_forward(const MlpLayout& L, const float* p, const __bf16* pb, const __bf16* X, int B, MlpActs& a,
                       float* out, hipStream_t st) {
  const int H = L.hidden;
  hipError_t e;
  Opnd x{X, L.in_pad, 1, B, L.in_pad, 1};
  Opnd w1{pb + L.W1, L.in_pad, 1, H, L.in_pad, 1};
  if ((e = gemm(x, w1, B, H, L.in_pad, p + L.b1, 1, 0, a.A1, H, a.A1b, H, st)) != hipSuccess) return e;
  Opnd a1{a.A1b, H, 1, B, H, 1};
  Opnd w2{pb + L.W2, H, 1, H, H, 1};
  if ((e = gemm(a1, w2, B, H, H, p + L.b2, 1, 0, a.A2, H, a.A2b, H, st)) != hipSuccess) return e;
  Opnd a2{a.A2b, H, 1, B, H, 1};
  Opnd w3{pb + L.W3, H, 1, H, H, 1};
  if ((e = gemm(a2, w3, B, H, H, p + L.b3, 1, 0, a.A3, H, nullptr, 0, st)) != hipSuccess) return e;
  k_mlp_head<<<(unsigned)((B + 3) / 4), 256, 0, st>>>(a.A3, pb + L.w4, p + L.b4, B, H, out);
  return hipGetLastError();
}

// Loss and gradient of a batch (after mlp_forward): grad (FP32, layout L).
hipError_t mlp_backward(const MlpLayout& L, const __bf16* pb, const __bf16* X, const float* y, int B, float tau,
                        MlpActs& a, const float* out, float* grad, float* loss, hipStream_t st) {
  const int H = L.hidden;
  hipError_t e;
  k_mlp_loss<<<1, 256, 0, st>>>(out, y, B, tau, a.g, loss);
  k_mlp_head_bwd<<<blocks(H), 256, 0, st>>>(a.A3, a.g, pb + L.w4, B, H, a.dZ, grad + L.w4, grad + L.b4);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // layer 3: dW3[h][k] = sum_b dZ3[b][h] A2[b][k]; dA2 = dZ3 W3
  Opnd dz_t{a.dZ, 1, H, H, B, 0};           // (h, b) -> dZ[b][h]
  Opnd a2_t{a.A2b, 1, H, H, B, 1};          // (k, b) -> A2[b][k]
  if ((e = gemm(dz_t, a2_t, H, H, B, nullptr, 0, 0, grad + L.W3, H, nullptr, 0, st)) != hipSuccess) return e;
  k_mlp_bias_grad<<<blocks(H), 256, 0, st>>>(a.dZ, B, H, grad + L.b3);
  Opnd dz{a.dZ, H, 1, B, H, 0};             // (b, h)
  Opnd w3_t{pb + L.W3, 1, H, H, H, 1};      // (k, h) -> W3[h][k]
  if ((e = gemm(dz, w3_t, B, H, H, nullptr, 0, 0, a.dZ2, H, nullptr, 0, st)) != hipSuccess) return e;
  k_mlp_relu_gate<<<blocks((int64_t)B * H), 256, 0, st>>>(a.dZ2, a.A2, (int64_t)B * H);
  // layer 2
  Opnd dz2_t{a.dZ2, 1, H, H, B, 0};
  Opnd a1_t{a.A1b, 1, H, H, B, 1};
  if ((e = gemm(dz2_t, a1_t, H, H, B, nullptr, 0, 0, grad + L.W2, H, nullptr, 0, st)) != hipSuccess) return e;
  k_mlp_bias_grad<<<blocks(H), 256, 0, st>>>(a.dZ2, B, H, grad + L.b2);
  Opnd dz2{a.dZ2, H, 1, B, H, 0};
  Opnd w2_t{pb + L.W2, 1, H, H, H, 1};
  if ((e = gemm(dz2, w2_t, B, H, H, nullptr, 0, 0, a.dZ, H, nullptr, 0, st)) != hipSuccess) return e;
  k_mlp_relu_gate<<<blocks((int64_t)B * H), 256, 0, st>>>(a.dZ, a.A1, (int64_t)B * H);
  // layer 1
  Opnd dz1_t{a.dZ, 1, H, H, B, 0};
  Opnd x_t{X, 1, L.in_pad, L.in_pad, B, 1};
  if ((e = gemm(dz1_t, x_t, H, L.in_pad, B, nullptr, 0, 0, grad + L.W1, L.in_pad, nullptr, 0, st)) != hipSuccess)
    return e;
  k_mlp_bias_grad<<<blocks(H), 256, 0, st>>>(a.dZ, B, H, grad + L.b1);
  return hipGetLastError();
}

hipError_t mlp_adam(float* p, __bf16* pb, const float* g, float* m, float* v, int64_t count, float lr, int step,
                    hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  k_mlp_adam<<<blocks(count), 256, 0, st>>>(p, pb, g, m, v, count, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* src, __bf16* dst, int64_t count, hipStream_t st) {
  k_to_bf16<<<blocks(count), 256, 0, st>>>(src, dst, count);
  return hipGetLastError();
}

}  // namespace adg
