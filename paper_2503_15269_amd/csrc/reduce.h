// Wavefront and workgroup reductions for gfx950 (wave64).
//
// Within a 16-lane DPP row the sum is formed with four DPP moves (quad
// permutations, half-row mirror, row mirror); the four row sums are then
// read with v_readlane and added in a fixed order, so every lane of every
// wave obtains the bitwise-same total. Across waves the per-wave totals go
// through LDS and are added in wave order. The result is deterministic.
//
// Dot products of float32 vectors sum the products in float64: the product
// of two float32 values is exact there, so only the float64 additions
// round, which is more accurate than a compensated float32 sum (Ogita, Rump
// and Oishi's Dot2, twice the float32 precision) and takes fewer
// instructions per term.
#pragma once

#include <hip/hip_runtime.h>

namespace btk {

// DPP control codes (GFX9 encoding).
constexpr int DPP_QUAD_1032 = 0xB1;  // lane ^ 1
constexpr int DPP_QUAD_2301 = 0x4E;  // lane ^ 2
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  long long u = __double_as_longlong(v);
  int lo = (int)(u & 0xffffffffll);
  int hi = (int)(u >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) |
                              (long long)(unsigned int)lo);
}

__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double readlane(double v, int l) {
  long long u = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), l);
  int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) |
                              (long long)(unsigned int)lo);
}

// ---------------------------------------------------------------- double
struct AccD {
  double s;
  __device__ __forceinline__ void zero() { s = 0.0; }
  __device__ __forceinline__ void add(double v) { s += v; }
  __device__ __forceinline__ void add_prod(double x, double y) {
    s = __fma_rn(x, y, s);
  }
  __device__ __forceinline__ void merge(const AccD& o) { s += o.s; }
  __device__ __forceinline__ double value() const { return s; }
  template <int CTRL>
  __device__ __forceinline__ AccD moved() const {
    AccD r;
    r.s = dpp<CTRL>(s);
    return r;
  }
  __device__ __forceinline__ AccD lane(int l) const {
    AccD r;
    r.s = readlane(s, l);
    return r;
  }
};

// ---------------------------------------- float products, float64 sums
// The product of two float32 values is exact in float64 (24 + 24 significant
// bits), so each term enters the sum unrounded: two conversions and a float64
// FMA per term, one float64 addition per merge.
struct AccX {
  double s;
  __device__ __forceinline__ void zero() { s = 0.0; }
  __device__ __forceinline__ void add(float v) { s += (double)v; }
  __device__ __forceinline__ void add_prod(float x, float y) {
    s = __fma_rn((double)x, (double)y, s);
  }
  __device__ __forceinline__ void merge(const AccX& o) { s += o.s; }
  __device__ __forceinline__ double value() const { return s; }
  template <int CTRL>
  __device__ __forceinline__ AccX moved() const {
    AccX r;
    r.s = dpp<CTRL>(s);
    return r;
  }
  __device__ __forceinline__ AccX lane(int l) const {
    AccX r;
    r.s = readlane(s, l);
    return r;
  }
};

template <typename T> struct AccOf;
template <> struct AccOf<double> { using type = AccD; };
template <> struct AccOf<float> { using type = AccX; };

// Sum over the 16 lanes of each DPP row; every lane of a row returns it.
template <typename A>
__device__ __forceinline__ A row16_sum(A v) {
  v.merge(v.template moved<DPP_QUAD_1032>());
  v.merge(v.template moved<DPP_QUAD_2301>());
  v.merge(v.template moved<DPP_ROW_HALF_MIRROR>());
  v.merge(v.template moved<DPP_ROW_MIRROR>());
  return v;
}

// Sum over the 64 lanes of a wave; every lane returns the same value.
template <typename A>
__device__ __forceinline__ A wave_sum(A v) {
  v.merge(v.template moved<DPP_QUAD_1032>());
  v.merge(v.template moved<DPP_QUAD_2301>());
  v.merge(v.template moved<DPP_ROW_HALF_MIRROR>());
  v.merge(v.template moved<DPP_ROW_MIRROR>());
  A t = v.lane(0);
  t.merge(v.lane(16));
  t.merge(v.lane(32));
  t.merge(v.lane(48));
  return t;
}

// Sum over the workgroup. ``slot`` is an LDS array of NT/64 entries that no
// thread reads or writes until the next barrier after this call returns.
template <int NT, typename A>
__device__ __forceinline__ A block_sum(A v, A* slot) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = v;
  __syncthreads();
  A t = slot[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) t.merge(slot[w]);
  return t;
}

}  // namespace btk
