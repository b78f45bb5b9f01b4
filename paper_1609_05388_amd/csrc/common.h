// Shared device/host definitions of the gfx950 ADAGIO library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace adg {

// Unit roundoff of FP32 and FP64 (round to nearest).
constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53

// Row tiling of the all-pairs screen: tiles of kTile x kTile pairs, inputs
// padded to a multiple of kTile rows and kChunk columns.
constexpr int kTile = 128;
constexpr int kChunk = 16;

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// FP32 values of a tile's point Gram in the screens' point-Gram cache.
constexpr int64_t kGcacheFloatsPerTile = (int64_t)kTile * kTile;
// Bytes of a tile's block in the precision-form screens' compact D^2 cache
// (one FP16 value per pair).
constexpr int64_t kDcacheBytesPerTile = (int64_t)kTile * kTile * 2;

// kNN screen: candidates kept per query and database split, and the most
// splits one query's keys may span.
constexpr int kKnnKeep = 32;
constexpr int kKnnMaxSplits = 32;
constexpr int kKnnQueries = 64;   // queries per screen workgroup

// One tile record of the screen: the largest upper bound on the squared
// distance ratio q = E^2 / D^2 in the tile with its pair, and the smallest
// lower bound with its pair.  Pairs are global point indices, i < j.
struct TileRec {
  float qhi;
  float qlo;
  int32_t ihi, jhi;
  int32_t ilo, jlo;
  int32_t pad0, pad1;
};

// One exactly re-evaluated pair.
struct PairVal {
  double v;      // eq. (2) distortion in FP64; -1 for identical points
  int32_t i, j;  // i < j
  int32_t side;  // +1 expansion, -1 contraction, 0 equal
  int32_t pad;
};

// Device-side state of one certificate, written by the finalising kernels.
struct CertDev {
  PairVal best;         // best exact pair so far
  PairVal second;       // runner-up among exactly evaluated pairs
  float thr_hi;         // emit a pair when its q upper bound >= thr_hi
  float thr_lo;         // ... or its q lower bound <= thr_lo
  uint32_t n_flagged;   // tiles that need the exact second pass
  uint32_t n_cand;      // candidate pairs emitted by that pass (may exceed capacity)
  double bound_rest;    // bound on every pair not re-evaluated
  int32_t n_seed;       // pairs evaluated while seeding the threshold
  float qhi_all;        // largest q upper bound over all pairs
  float qlo_all;        // smallest q lower bound over all pairs
  int32_t pad;
};

__host__ __device__ inline bool pair_better(double va, int32_t ia, int32_t ja, double vb, int32_t ib, int32_t jb) {
  if (va != vb) return va > vb;
  if (ia != ib) return ia < ib;
  return ja < jb;
}

}  // namespace adg
