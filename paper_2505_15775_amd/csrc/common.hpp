// Device-side helpers shared by the ALM-BM kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace almbm {

constexpr int kBlock = 256;          // threads per block for every row kernel
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kNumXcd = 8;           // MI355X: 8 XCDs, blocks dispatched round robin

// bfloat16 storage: 16 high bits of an IEEE binary32.
struct bf16 {
  uint16_t bits;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// Round a binary32 to the nearest bfloat16, ties to even; NaN stays NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<uint16_t>((u >> 16) | 0x40u);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return static_cast<uint16_t>(u >> 16);
}

// Storage type -> arithmetic type.
template <typename T> struct Acc { using type = float; };
template <> struct Acc<double> { using type = double; };

template <typename T> __device__ __forceinline__ typename Acc<T>::type to_acc(T v) { return v; }
template <> __device__ __forceinline__ float to_acc<bf16>(bf16 v) { return bf16_to_f32(v.bits); }

template <typename T> __device__ __forceinline__ T from_acc(typename Acc<T>::type v) { return v; }
template <> __device__ __forceinline__ bf16 from_acc<bf16>(float v) { return bf16{f32_to_bf16(v)}; }

// Value rounded to storage precision and back (what a store then load would give).
template <typename T> __device__ __forceinline__ typename Acc<T>::type round_st(typename Acc<T>::type v) {
  return to_acc<T>(from_acc<T>(v));
}

// ---- row fragments: LPR lanes hold one row of r <= LPR*VEC elements ----------
//
// Lane l of a row group owns columns [l*VEC, l*VEC+VEC).  FULL means
// r == LPR*VEC, so a lane's slice is contiguous and aligned to VEC*sizeof(T)
// bytes and is moved with one vector access.

template <int BYTES> struct VecWord;
template <> struct VecWord<2> { using type = uint16_t; };
template <> struct VecWord<4> { using type = uint32_t; };
template <> struct VecWord<8> { using type = uint2; };
template <> struct VecWord<16> { using type = uint4; };
template <> struct VecWord<32> { struct type { uint4 a, b; }; };
template <> struct VecWord<64> { struct type { uint4 a, b, c, d; }; };

template <typename T, int VEC, bool FULL>
__device__ __forceinline__ void load_frag(const T* __restrict__ row, int lane, int r,
                                          typename Acc<T>::type (&out)[VEC]) {
  if constexpr (FULL) {
    using W = typename VecWord<VEC * sizeof(T)>::type;
    W w = *reinterpret_cast<const W*>(row + lane * VEC);
    const T* e = reinterpret_cast<const T*>(&w);
#pragma unroll
    for (int v = 0; v < VEC; ++v) out[v] = to_acc<T>(e[v]);
  } else {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      int c = lane * VEC + v;
      out[v] = (c < r) ? to_acc<T>(row[c]) : typename Acc<T>::type(0);
    }
  }
}

template <typename T, int VEC, bool FULL>
__device__ __forceinline__ void store_frag(T* __restrict__ row, int lane, int r,
                                           const typename Acc<T>::type (&in)[VEC]) {
  if constexpr (FULL) {
    using W = typename VecWord<VEC * sizeof(T)>::type;
    W w;
    T* e = reinterpret_cast<T*>(&w);
#pragma unroll
    for (int v = 0; v < VEC; ++v) e[v] = from_acc<T>(in[v]);
    *reinterpret_cast<W*>(row + lane * VEC) = w;
  } else {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      int c = lane * VEC + v;
      if (c < r) row[c] = from_acc<T>(in[v]);
    }
  }
}

// Sum over the LPR lanes of a row group (all lanes of the group get the sum).
template <int LPR, typename V>
__device__ __forceinline__ V group_sum(V x) {
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, LPR);
  return x;
}

template <typename V>
__device__ __forceinline__ V wave_sum(V x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// Deterministic block sum of NS doubles per thread; result written by thread 0
// to out[0..NS).  Fixed order: lanes by butterfly, then waves in index order.
template <int NS>
__device__ __forceinline__ void block_sum_store(double (&acc)[NS], double* __restrict__ out) {
  __shared__ double red[kBlock / kWave][NS];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double v = wave_sum(acc[s]);
    if (lane == 0) red[wave][s] = v;
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) t += red[w][threadIdx.x];
    out[threadIdx.x] = t;
  }
}

// Rows owned by this block: the row range is split into gridDim.x contiguous
// chunks and blocks are renumbered so that the blocks the hardware sends to one
// XCD (blockIdx % 8 equal) own one contiguous eighth of the rows; neighbour rows
// of banded or mesh-like patterns then stay in that XCD's L2.
struct RowChunk {
  long lo, hi;
};
__device__ __forceinline__ RowChunk row_chunk(long n) {
  const long nb = gridDim.x;
  long vb = blockIdx.x;
  if (nb % kNumXcd == 0) {
    const long per = nb / kNumXcd;
    vb = (blockIdx.x % kNumXcd) * per + blockIdx.x / kNumXcd;
  }
  const long chunk = (n + nb - 1) / nb;
  long lo = vb * chunk;
  long hi = lo + chunk;
  if (lo > n) lo = n;
  if (hi > n) hi = n;
  return {lo, hi};
}

// Counter-based uniform in [-1, 1) from (seed, index): the SplitMix64 output
// function (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) applied to seed * golden + index.
__device__ __forceinline__ double counter_uniform(uint64_t seed, uint64_t idx) {
  uint64_t z = seed * 0x9e3779b97f4a7c15ull + (idx + 1) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z = z ^ (z >> 31);
  return static_cast<double>(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

}  // namespace almbm
