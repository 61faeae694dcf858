// Sparse row product shared by the row kernels.
#pragma once

#include "kernels.hpp"

namespace almbm {

// p = d_i x_i + sum_k S_ik x_{col k} for the row group's slice of columns;
// X rows have stride r.  Two neighbours per step so that both row gathers are
// in flight together.
template <typename T, int LPR, int VEC, bool FULL>
__device__ __forceinline__ void spmm_row(const Cost<typename Acc<T>::type>& C, long i, int lane, int r,
                                         const T* __restrict__ X,
                                         const typename Acc<T>::type (&xi)[VEC],
                                         typename Acc<T>::type (&p)[VEC]) {
  using V = typename Acc<T>::type;
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
    k0 = k1 = 0;
  }
  long k = k0;
  // two neighbours per step: both gathers are issued before either is used
  for (; k + 1 < k1; k += 2) {
    const int j0 = C.ci[k], j1 = C.ci[k + 1];
    const V c0 = C.cv[k], c1 = C.cv[k + 1];
    V x0[VEC], x1[VEC];
    load_frag<T, VEC, FULL>(X + (long)j0 * r, lane, r, x0);
    load_frag<T, VEC, FULL>(X + (long)j1 * r, lane, r, x1);
#pragma unroll
    for (int v = 0; v < VEC; ++v) p[v] += c0 * x0[v] + c1 * x1[v];
  }
  if (k < k1) {
    const int j0 = C.ci[k];
    const V c0 = C.cv[k];
    V x0[VEC];
    load_frag<T, VEC, FULL>(X + (long)j0 * r, lane, r, x0);
#pragma unroll
    for (int v = 0; v < VEC; ++v) p[v] += c0 * x0[v];
  }
}

}  // namespace almbm
