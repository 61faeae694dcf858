// Random-row gather probe: the rate at which the chip serves independent
// gathers of whole rows from a table in HBM, the access that bounds the sparse
// cost product (every nonzero of C gathers one row of the factor).  Lane groups
// of L lanes read rows idx[k] (8 bytes per lane, kUnroll rows in flight per
// group, like the product's row loop) and keep a running sum so that no load
// is dead; every thread writes its sum.
#include <hip/hip_runtime.h>

#include <string>

#include "alm_bm.h"
#include "api_internal.hpp"
#include "common.hpp"

using namespace almbm;

namespace {

constexpr int kProbeBlocks = 4096;
constexpr int kProbeUnroll = 4;

template <int L>
__global__ void __launch_bounds__(kBlock)
k_gather_probe(const uint2* __restrict__ table, const int32_t* __restrict__ idx, long count, float* __restrict__ out) {
  const int lane = threadIdx.x % L;
  const long grp = ((long)blockIdx.x * kBlock + threadIdx.x) / L;
  const long ngrp = (long)gridDim.x * kBlock / L;
  float acc = 0.f;
  long k = grp;
  for (; k + (kProbeUnroll - 1) * ngrp < count; k += kProbeUnroll * ngrp) {
    uint2 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = table[(long)idx[k + u * ngrp] * L + lane];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc += __uint_as_float(v[u].x) + __uint_as_float(v[u].y);
  }
  for (; k < count; k += ngrp) {
    const uint2 v = table[(long)idx[k] * L + lane];
    acc += __uint_as_float(v.x) + __uint_as_float(v.y);
  }
  out[(long)blockIdx.x * kBlock + threadIdx.x] = acc;
}

}  // namespace

extern "C" int64_t alm_bm_gather_probe_out_size(void) { return (int64_t)kProbeBlocks * kBlock; }

extern "C" alm_bm_status alm_bm_gather_probe(const void* table, int64_t rows, int32_t row_bytes, const int32_t* idx,
                                             int64_t count, float* out, hipStream_t st) {
  if (!table || !idx || !out || rows < 1 || count < 0)
    return set_error(ALM_BM_ERR_INVALID_ARG, "gather_probe: null pointer or bad size");
  const dim3 grid(kProbeBlocks), block(kBlock);
  const uint2* t = static_cast<const uint2*>(table);
  switch (row_bytes) {
    case 8: hipLaunchKernelGGL((k_gather_probe<1>), grid, block, 0, st, t, idx, count, out); break;
    case 16: hipLaunchKernelGGL((k_gather_probe<2>), grid, block, 0, st, t, idx, count, out); break;
    case 32: hipLaunchKernelGGL((k_gather_probe<4>), grid, block, 0, st, t, idx, count, out); break;
    case 64: hipLaunchKernelGGL((k_gather_probe<8>), grid, block, 0, st, t, idx, count, out); break;
    case 128: hipLaunchKernelGGL((k_gather_probe<16>), grid, block, 0, st, t, idx, count, out); break;
    case 256: hipLaunchKernelGGL((k_gather_probe<32>), grid, block, 0, st, t, idx, count, out); break;
    default: return set_error(ALM_BM_ERR_INVALID_ARG, "gather_probe: row_bytes must be 8, 16, 32, 64, 128 or 256");
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ALM_BM_ERR_HIP, std::string("gather_probe: ") + hipGetErrorString(e));
  return ALM_BM_OK;
}
