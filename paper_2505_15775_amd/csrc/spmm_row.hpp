// Sparse row product shared by the row kernels.
#pragma once

#include "kernels.hpp"

namespace almbm {

constexpr int kUnroll = 4;  // neighbour rows gathered together per step

// p = d_i x_i + sum_k S_ik x_{col k} for the row group's slice of columns;
// X rows have stride r.  The neighbour loop issues kUnroll row gathers before
// consuming any of them and fetches the next indices while they are in flight,
// so that each wave keeps several independent HBM/Infinity-Cache requests
// outstanding (the kernel is bound by gather latency, not by arithmetic).
template <typename T, int LPR, int VEC, bool FULL>
__device__ __forceinline__ void spmm_row(const Cost<typename Acc<T>::type>& C, long i, int lane, int r,
                                         const T* __restrict__ X,
                                         const typename Acc<T>::type (&xi)[VEC],
                                         typename Acc<T>::type (&p)[VEC]) {
  using V = typename Acc<T>::type;
  constexpr int U = kUnroll;
  const V di = C.dg ? C.dg[i] : V(0);
#pragma unroll
  for (int v = 0; v < VEC; ++v) p[v] = di * xi[v];
  long k0, k1;
  if (C.ell > 0) {
    k0 = i * (long)C.ell;
    k1 = k0 + C.ell;
  } else if (C.rp) {
    k0 = C.rp[i];
    k1 = C.rp[i + 1];
  } else {
    return;
  }
  if (k0 >= k1) return;
  if (C.nh > 0 && k1 - k0 > C.hthr) {  // hub row: sum precomputed by k_hub_rows
    const V* hs = C.hsum + (long)hub_index(C, i) * r;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const int c = lane * VEC + v;
      if (FULL || c < r) p[v] += hs[c];
    }
    return;
  }
  // indices and values of the first chunk; entries past the row end point at
  // row i itself with weight 0 (in bounds, no branch in the gather)
  int j[U];
  V c[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long k = k0 + u;
    j[u] = (k < k1) ? C.ci[k] : (int)i;
    c[u] = (k < k1) ? C.cv[k] : V(0);
  }
  for (long k = k0; k < k1; k += U) {
    V x[U][VEC];
#pragma unroll
    for (int u = 0; u < U; ++u) load_frag<T, VEC, FULL>(X + (long)j[u] * r, lane, r, x[u]);
    V cc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cc[u] = c[u];
    // next chunk's indices while the gathers are outstanding
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long kn = k + U + u;
      j[u] = (kn < k1) ? C.ci[kn] : (int)i;
      c[u] = (kn < k1) ? C.cv[kn] : V(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < VEC; ++v) p[v] += cc[u] * x[u][v];
  }
}

// Row-partial accumulators spread over the LPR lanes of a row group: lane l
// keeps the slots s with s % LPR == l, so each lane holds ceil(NS/LPR) doubles
// instead of NS.  add() takes a value every lane of the group agrees on.
template <int NS, int LPR>
struct SplitAcc {
  static constexpr int K = (NS + LPR - 1) / LPR;
  double a[K];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int q = 0; q < K; ++q) a[q] = 0.0;
  }
  __device__ __forceinline__ void add(int lane, int s, double v) {
    if (LPR == 1) {
      a[s] += v;
    } else {
      a[s / LPR] += (lane == s % LPR) ? v : 0.0;
    }
  }
  // Deterministic block total of every slot into out[0..NS): per-thread slots
  // to LDS, then slot s summed over threads t = s % LPR, s % LPR + LPR, ... in order.
  __device__ __forceinline__ void block_store(int lane, double* __restrict__ out) {
    __shared__ double buf[kBlock][K];
#pragma unroll
    for (int q = 0; q < K; ++q) buf[threadIdx.x][q] = a[q];
    __syncthreads();
    if (threadIdx.x < NS) {
      const int s = threadIdx.x;
      const int l = s % LPR, q = s / LPR;
      double t = 0.0;
      for (int th = l; th < kBlock; th += LPR) t += buf[th][q];
      out[s] = t;
    }
  }
};

// Tile (lanes per row, columns per lane) for a rank r.  `variant` selects an
// alternative tile for the same r (autotuner); 0 is the default.
#define ALMBM_DISPATCH_DIAG(T, FN, ...)                                                   \
  do {                                                                                    \
    if constexpr (sizeof(T) == 8) {                                                       \
      if (r <= 4) FN<T, 4, 1>(__VA_ARGS__);                                               \
      else if (r <= 8) { if (variant == 1) FN<T, 4, 2>(__VA_ARGS__); else FN<T, 8, 1>(__VA_ARGS__); } \
      else if (r <= 16) {                                                                 \
        if (variant == 1) FN<T, 16, 1>(__VA_ARGS__);                                      \
        else if (variant == 2) FN<T, 4, 4>(__VA_ARGS__);                                  \
        else FN<T, 8, 2>(__VA_ARGS__);                                                    \
      } else if (r <= 32) { if (variant == 1) FN<T, 16, 2>(__VA_ARGS__); else FN<T, 8, 4>(__VA_ARGS__); } \
      else if (r <= 64) FN<T, 16, 4>(__VA_ARGS__);                                        \
      else FN<T, 32, 4>(__VA_ARGS__);                                                     \
    } else if constexpr (sizeof(T) == 4) {                                                \
      if (r <= 4) FN<T, 4, 1>(__VA_ARGS__);                                               \
      else if (r <= 8) { if (variant == 1) FN<T, 8, 1>(__VA_ARGS__); else FN<T, 4, 2>(__VA_ARGS__); } \
      else if (r <= 16) {                                                                 \
        if (variant == 1) FN<T, 8, 2>(__VA_ARGS__);                                       \
        else if (variant == 2) FN<T, 2, 8>(__VA_ARGS__);                                  \
        else FN<T, 4, 4>(__VA_ARGS__);                                                    \
      } else if (r <= 32) { if (variant == 1) FN<T, 4, 8>(__VA_ARGS__); else FN<T, 8, 4>(__VA_ARGS__); } \
      else if (r <= 64) FN<T, 16, 4>(__VA_ARGS__);                                        \
      else FN<T, 32, 4>(__VA_ARGS__);                                                     \
    } else {                                                                              \
      if (r <= 4) FN<T, 2, 2>(__VA_ARGS__);                                               \
      else if (r <= 8) { if (variant == 1) FN<T, 1, 8>(__VA_ARGS__); else FN<T, 2, 4>(__VA_ARGS__); } \
      else if (r <= 16) {                                                                 \
        if (variant == 1) FN<T, 4, 4>(__VA_ARGS__);                                       \
        else if (variant == 2) FN<T, 1, 16>(__VA_ARGS__);                                 \
        else FN<T, 2, 8>(__VA_ARGS__);                                                    \
      } else if (r <= 32) { if (variant == 1) FN<T, 8, 4>(__VA_ARGS__); else FN<T, 4, 8>(__VA_ARGS__); } \
      else if (r <= 64) FN<T, 8, 8>(__VA_ARGS__);                                         \
      else FN<T, 16, 8>(__VA_ARGS__);                                                     \
    }                                                                                     \
  } while (0)

}  // namespace almbm
