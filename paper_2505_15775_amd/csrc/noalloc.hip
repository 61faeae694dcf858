// Objective and gradient of eq. (AL-BM) for callers that cannot allocate
// device memory: no handle, and the per-block partial sums of the fused row
// kernel live in a fixed static device array instead of a handle's workspace.
// The kernels are the handle path's (k_objgrad_diag and its fixed-order
// finalize), launched with the same default grid, so the results are the ones
// alm_bm_objective_grad gives on a handle with default tiles.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "alm_bm.h"
#include "api_internal.hpp"
#include "launch.hpp"

using namespace almbm;

namespace {

// Largest grid row_blocks() returns, hence the most partial-sum rows a call
// needs; every n in 1..2^31-1 maps to at most this many blocks.
constexpr int kScratchBlocks = 4096;
constexpr size_t kPartDoubles = (size_t)kScratchBlocks * NUM_P;
constexpr size_t kScalarDoubles = (sizeof(DevScalars) + sizeof(double) - 1) / sizeof(double);
constexpr size_t kScratchDoubles = kPartDoubles + kScalarDoubles;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
double* g_dev_ptr[kMaxDevices] = {};

}  // namespace

// Per-GPU scratch: kScratchBlocks x NUM_P partial sums, then one DevScalars
// block for the finalize (about 0.5 MB; every GPU the library runs on holds its
// own copy until the process ends).  Host code never uses this name as an
// address: it passes the pointer hipGetSymbolAddress returned for the device.
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on the current device, resolved once per device
// (no allocation, no stream work).
static alm_bm_status scratch_ptr(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(ALM_BM_ERR_HIP, std::string("noalloc: hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(ALM_BM_ERR_UNSUPPORTED, "noalloc: device index >= 64");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_dev_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(ALM_BM_ERR_HIP, std::string("noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_dev_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_dev_ptr[dev];
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_objective_grad_noalloc(const alm_bm_problem_desc* desc, int32_t r,
                                                       const double* R, const double* y, double sigma, double* f,
                                                       double* G, double* Av, hipStream_t st) {
  if (!desc || !R || !y || !f) return set_error(ALM_BM_ERR_INVALID_ARG, "objective_grad_noalloc: null argument");
  const alm_bm_problem_desc& d = *desc;
  if (d.n <= 0 || d.n > INT32_MAX) return set_error(ALM_BM_ERR_INVALID_ARG, "objective_grad_noalloc: n out of range");
  if (r < 1 || r > kMaxR) return set_error(ALM_BM_ERR_INVALID_ARG, "objective_grad_noalloc: r must be in 1..128");
  if (d.cons_kind != ALM_BM_CONS_DIAG)
    return set_error(ALM_BM_ERR_UNSUPPORTED, "objective_grad_noalloc: only the DIAG constraint family");
  if (d.precision != ALM_BM_F64)
    return set_error(ALM_BM_ERR_UNSUPPORTED, "objective_grad_noalloc: only ALM_BM_F64 storage");
  if (d.j_coef != 0.0) return set_error(ALM_BM_ERR_UNSUPPORTED, "objective_grad_noalloc: cost with a -J term");
  if (d.m != d.n || !d.b) return set_error(ALM_BM_ERR_INVALID_ARG, "objective_grad_noalloc: DIAG needs m = n and b");
  if (d.nnz < 0 || d.nnz > INT32_MAX || (d.nnz > 0 && (!d.col_idx || !d.val)))
    return set_error(ALM_BM_ERR_INVALID_ARG, "objective_grad_noalloc: nnz out of range or col_idx/val null");
  if (d.ell_width < 0) return set_error(ALM_BM_ERR_INVALID_ARG, "objective_grad_noalloc: ell_width < 0");
  if (d.ell_width > 0 && d.nnz != d.n * (int64_t)d.ell_width)
    return set_error(ALM_BM_ERR_INVALID_ARG, "objective_grad_noalloc: ELL needs nnz = n * ell_width");
  if (d.ell_width == 0 && d.nnz > 0 && !d.row_ptr)
    return set_error(ALM_BM_ERR_INVALID_ARG, "objective_grad_noalloc: CSR needs row_ptr");
  const int nblk = row_blocks(d.n);
  if (nblk > kScratchBlocks)
    return set_error(ALM_BM_ERR_INVALID_ARG, "objective_grad_noalloc: grid larger than the scratch array");
  double* base = nullptr;
  const alm_bm_status s = scratch_ptr(&base);
  if (s < 0) return s;
  Cost<double> C{d.n, d.ell_width > 0 ? nullptr : (d.nnz ? d.row_ptr : nullptr), d.col_idx, d.val, d.ell_width,
                 d.diag};
  if (d.nnz == 0) C.rp = nullptr, C.ell = 0;
  double* part = base;
  DevScalars* sc = reinterpret_cast<DevScalars*>(base + kPartDoubles);
  // every block stores all NUM_P of its partial slots and the finalize (mode 0)
  // only writes the scalar block, so nothing in the scratch needs clearing
  launch_objgrad_diag<double>(C, r, 0, R, y, d.b, sigma, G, Av, part, nullptr, 0, BlockTab{}, nblk, st);
  launch_fin_objgrad(part, nblk, sc, sigma, 0, f, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return set_error(ALM_BM_ERR_HIP, std::string("objective_grad_noalloc: launch: ") + hipGetErrorString(e));
  return ALM_BM_OK;
}
