// Steps a4-a5: the JL matrix S of Lemma 1 / Algorithm 1 and the map
// Pi = [P ; S - (S P^T) P] (Algorithm 1 with Q = I - P^T P from the proof of
// Theorem 2; floor(r/2) / ceil(r/2) split of Sec. 4.1).
//
// S's entries are +-1/sqrt(k), drawn from a fixed infinite sign matrix B:
// entry (a, l) is the top bit of output number a * 2^32 + l + 1 of a
// SplitMix64 generator seeded with `seed` (Steele, Lea & Flood, OOPSLA 2014:
// state advanced by 0x9E3779B97F4A7C15, outputs passed through the published
// 64-bit finaliser).  Counter-based, so every entry is generated independently
// and rows are nested across k.
#include "common.h"
#include "kernels.h"

namespace adg {

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t t) {
  uint64_t z = seed + t * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// S[a][l] = (bit 63 of output (a << 32 | l) + 1 is 0 ? +1 : -1) / sqrt(k)
__global__ void k_jl_signs(uint64_t seed, int64_t k, int64_t d, double inv_sqrt_k, double* __restrict__ S) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= k * d) return;
  const uint64_t a = (uint64_t)(e / d), l = (uint64_t)(e % d);
  const uint64_t z = splitmix64_at(seed, ((a << 32) | l) + 1ull);
  S[e] = (z >> 63) ? -inv_sqrt_k : inv_sqrt_k;
}

// Pi[a][l] = fl32(Vt[a][l]) for a < rows (the principal rows P).
__global__ void k_copy_rows(const double* __restrict__ Vt, int64_t rows, int64_t d, float* __restrict__ Pi,
                            double* __restrict__ Pi64) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * d) return;
  const double v = Vt[e];
  Pi[e] = (float)v;
  if (Pi64) Pi64[e] = v;
}

hipError_t launch_jl_signs(uint64_t seed, int64_t k, int64_t d, double* S, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  k_jl_signs<<<(unsigned)((k * d + 255) / 256), 256, 0, st>>>(seed, k, d, 1.0 / sqrt((double)k), S);
  return hipGetLastError();
}

hipError_t launch_copy_rows(const double* Vt, int64_t rows, int64_t d, float* Pi, double* Pi64, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  k_copy_rows<<<(unsigned)((rows * d + 255) / 256), 256, 0, st>>>(Vt, rows, d, Pi, Pi64);
  return hipGetLastError();
}

}  // namespace adg
