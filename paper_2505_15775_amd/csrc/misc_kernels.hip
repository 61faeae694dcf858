// Scalar finalisation (deterministic fixed-order reductions), the quartic step
// rule, the factor update and the FP64 dual update.
#include <math.h>

#include "kernels.hpp"
#include "quartic.hpp"

namespace almbm {

// ---- deterministic reduction of per-block partials ---------------------------
// part is [nb][NS]; thread t sums blocks t, t+256, ... in order, then the block
// tree is fixed, so the total does not depend on timing.
template <int NS>
__device__ void reduce_partials(const double* __restrict__ part, int b0, int b1, int stride, double* __restrict__ out) {
  double acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = 0.0;
  for (int bi = b0 + threadIdx.x; bi < b1; bi += kBlock) {
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] += part[(long)bi * stride + s];
  }
  __shared__ double res[NS];
  block_sum_store<NS>(acc, res);
  __syncthreads();
  if (threadIdx.x < NS) out[threadIdx.x] = res[threadIdx.x];
  __syncthreads();
}

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// ---- finalize kernels (one block) ------------------------------------------------

// Objective totals of the DIAG family.  mode 0: API call, writes *f_out.
// mode 1: inner loop step 1 -- after max_inner steps stop (flag 2), else the
// stop test ||G|| ||R|| <= tol (1 + |<C,RR^T>|) (flag 1), else count the step.
// One block per instance (blockIdx.x; a single instance without a table).
__global__ void __launch_bounds__(kBlock)
k_fin_objgrad(const double* __restrict__ part, int nb, DevScalars* __restrict__ sc_base, double sigma, int mode,
              double* __restrict__ f_out, BlockTab tab) {
  const int q = blockIdx.x;
  DevScalars* sc = sc_base + q;
  if (mode == 1 && sc->flag) return;
  int b0, b1;
  inst_blocks(tab, q, nb, b0, b1);
  __shared__ double tot[NUM_P];
  reduce_partials<NUM_P>(part, b0, b1, NUM_P, tot);
  if (threadIdx.x != 0) return;
  if (f_out) f_out += q;
  for (int s = 0; s < NUM_P; ++s) sc->tot[s] = tot[s];
  const double f = tot[P_C0] + tot[P_YBMA] + 0.5 * sigma * tot[P_EE];
  sc->f = f;
  if (!finite(f) || !finite(tot[P_GG])) sc->numeric_error = 1;
  if (f_out) *f_out = f;
  if (mode == 1) {
    const double lhs = sqrt(tot[P_GG]) * sqrt(tot[P_RR]);
    if (sc->iter >= sc->max_inner) {
      sc->flag = 2;
    } else if (lhs <= sc->tol * (1.0 + fabs(tot[P_C0])) || !finite(lhs)) {
      sc->flag = 1;
    } else {
      sc->iter += 1;
    }
  }
}

// Step rule: reduce the <G, CG> partials into tot[P_C2], form the quartic and
// pick t.  mode 0: API (coeffs/t to the given pointers).  mode 1: inner loop.
__global__ void __launch_bounds__(kBlock)
k_fin_step(const double* __restrict__ part_c2, int nb, int c2_stride, DevScalars* __restrict__ sc_base, double sigma,
           double j_extra_c2, int mode, double* __restrict__ coeffs_out, double* __restrict__ t_out, BlockTab tab) {
  const int q = blockIdx.x;
  DevScalars* sc = sc_base + q;
  if (mode == 1 && sc->flag) return;
  int b0, b1;
  inst_blocks(tab, q, nb, b0, b1);
  __shared__ double c2[1];
  if (part_c2) reduce_partials<1>(part_c2, b0, b1, c2_stride, c2);
  if (threadIdx.x != 0) return;
  if (part_c2) sc->tot[P_C2] = c2[0] + j_extra_c2;
  double k[5];
  quartic_coeffs(sc->tot, sigma, k);
  for (int s = 0; s < 5; ++s) sc->coeffs[s] = k[s];
  double t = (sc->step_rule == 1 && mode == 1) ? sc->eta_fixed : quartic_argmin(k);
  if (!finite(t)) {
    t = 0.0;
    sc->numeric_error = 1;
  }
  sc->t = t;
  if (coeffs_out)
    for (int s = 0; s < 5; ++s) coeffs_out[s] = k[s];
  if (t_out) *t_out = t;
}

// Full reduction of all NUM_P partials (API line search), then the step.
__global__ void __launch_bounds__(kBlock)
k_fin_ls(const double* __restrict__ part, int nb, DevScalars* __restrict__ sc, double sigma,
         double* __restrict__ coeffs_out, double* __restrict__ t_out) {
  __shared__ double tot[NUM_P];
  reduce_partials<NUM_P>(part, 0, nb, NUM_P, tot);
  if (threadIdx.x != 0) return;
  for (int s = 0; s < NUM_P; ++s) sc->tot[s] = tot[s];
  double k[5];
  quartic_coeffs(sc->tot, sigma, k);
  const double t = quartic_argmin(k);
  for (int s = 0; s < 5; ++s) sc->coeffs[s] = k[s];
  sc->t = t;
  if (coeffs_out)
    for (int s = 0; s < 5; ++s) coeffs_out[s] = k[s];
  if (t_out) *t_out = t;
}

// R <- R - t G (elementwise, storage precision), skipped once the flag is set.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_update(long len, T* __restrict__ R, const T* __restrict__ G, const DevScalars* __restrict__ sc, int use_flag) {
  using V = typename Acc<T>::type;
  if (use_flag && sc->flag) return;
  const V t = static_cast<V>(sc->t);
  const long stride = (long)gridDim.x * kBlock;
  for (long idx = (long)blockIdx.x * kBlock + threadIdx.x; idx < len; idx += stride) {
    R[idx] = from_acc<T>(to_acc<T>(R[idx]) - t * to_acc<T>(G[idx]));
  }
}

// y_out = y_in - sigma (Av - b); partials {||Av - b||^2, b^T y_out}.
__global__ void __launch_bounds__(kBlock)
k_dual(long m, const double* __restrict__ Av, const double* __restrict__ b, const double* __restrict__ y_in,
       double* __restrict__ y_out, double sigma, double sigma_tail, double* __restrict__ part, BlockTab tab) {
  double acc[2] = {0.0, 0.0};
  long i0, i1, step;
  if (tab.inst) {
    const Rows rw = rows_of(m, tab);
    i0 = rw.lo + threadIdx.x;
    i1 = rw.hi;
    step = kBlock;
  } else {
    i0 = (long)blockIdx.x * kBlock + threadIdx.x;
    i1 = m;
    step = (long)gridDim.x * kBlock;
  }
  for (long i = i0; i < i1; i += step) {
    const double e = Av[i] - b[i];
    const double yn = y_in[i] - (i == 0 ? sigma : sigma_tail) * e;
    if (y_out) y_out[i] = yn;
    acc[0] += e * e;
    acc[1] += b[i] * yn;
  }
  block_sum_store<2>(acc, part + (long)blockIdx.x * 2);
}

__global__ void __launch_bounds__(kBlock)
k_fin_dual(const double* __restrict__ part, int nb, DevScalars* __restrict__ sc_base, double bnorm,
           const double* __restrict__ bnorms, double* __restrict__ pinf_out, BlockTab tab) {
  const int q = blockIdx.x;
  DevScalars* sc = sc_base + q;
  if (bnorms) bnorm = bnorms[q];
  int b0, b1;
  inst_blocks(tab, q, nb, b0, b1);
  __shared__ double tot[2];
  reduce_partials<2>(part, b0, b1, 2, tot);
  if (threadIdx.x != 0) return;
  if (pinf_out) pinf_out += q;
  sc->res2 = tot[0];
  sc->pinf = sqrt(tot[0]) / (1.0 + bnorm);
  sc->dobj = tot[1];
  if (!finite(sc->pinf) || !finite(sc->dobj)) sc->numeric_error = 1;
  if (pinf_out) *pinf_out = sc->pinf;
}

// Start of an inner solve: clear the flag and counters (a kernel, not a memset,
// so that it can sit inside a captured graph).
__global__ void k_inner_reset(DevScalars* sc, double tol, int max_inner, int step_rule, double eta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->flag = 0;
    sc->iter = 0;
    sc->numeric_error = 0;
    sc->tol = tol;
    sc->max_inner = max_inner;
    sc->step_rule = step_rule;
    sc->eta_fixed = eta;
  }
}

// Batched reset: instance q runs (flag 0) when active[q], else is frozen (flag 3).
__global__ void k_inner_reset_batch(DevScalars* sc, int count, const double* __restrict__ tols,
                                    const int32_t* __restrict__ active, int max_inner, int step_rule, double eta) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  sc[q].flag = active[q] ? 0 : 3;
  sc[q].iter = 0;
  sc[q].numeric_error = 0;
  sc[q].tol = tols[q];
  sc[q].max_inner = max_inner;
  sc[q].step_rule = step_rule;
  sc[q].eta_fixed = eta;
}

// Batched helpers: y <- ybuf on the rows of active instances; column c_q of R
// (row stride rs) <- scale_q v on the rows of instance q where scale_q >= 0.
__global__ void __launch_bounds__(kBlock)
k_copy_active(long m, const double* __restrict__ src, double* __restrict__ dst, const int32_t* __restrict__ active,
              BlockTab tab) {
  const Rows rw = rows_of(m, tab);
  if (!active[rw.inst]) return;
  for (long i = rw.lo + threadIdx.x; i < rw.hi; i += kBlock) dst[i] = src[i];
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_fill_column(long n, int rs, T* __restrict__ R, const double* __restrict__ v, const int32_t* __restrict__ col,
              const double* __restrict__ scale, BlockTab tab) {
  const Rows rw = rows_of(n, tab);
  const double s = scale[rw.inst];
  if (!(s >= 0.0)) return;
  const int c = col[rw.inst];
  R += row_base(tab, rw.inst);
  for (long i = rw.lo + threadIdx.x; i < rw.hi; i += kBlock)
    R[i * rs + c] = from_acc<T>(static_cast<typename Acc<T>::type>(s * v[i]));
}

// Batched factor re-layout: for every row i of instance q (blocks of the full
// table), dst[nb_q + i ns_q + c] = src[ob_q + i os_q + c] for c < nc_q and 0
// for nc_q <= c < ns_q.  src and dst must not overlap.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_restride_batch(BlockTab tab, const T* __restrict__ src, T* __restrict__ dst, const int64_t* __restrict__ ob,
                 const int32_t* __restrict__ os, const int64_t* __restrict__ nbase, const int32_t* __restrict__ ns,
                 const int32_t* __restrict__ nc) {
  const int q = tab.inst[blockIdx.x];
  const long lo = tab.lo[blockIdx.x], hi = tab.hi[blockIdx.x];
  const int w = ns[q], wo = os[q], c0 = nc[q];
  const long len = (hi - lo) * (long)w;
  for (long e = threadIdx.x; e < len; e += kBlock) {
    const long i = lo + e / w;
    const int c = (int)(e % w);
    dst[nbase[q] + i * w + c] = c < c0 ? src[ob[q] + i * wo + c] : from_acc<T>(typename Acc<T>::type(0));
  }
}

// R[:, c] <- scale * v (row stride rs), one instance.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_set_column(long n, int rs, int c, T* __restrict__ R, const double* __restrict__ v, double scale) {
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    R[i * rs + c] = from_acc<T>(static_cast<typename Acc<T>::type>(scale * v[i]));
}

// Copy with change of row stride: dst (n x rd) gets the first nc columns of src
// (row stride ss); column nc of dst (when nc < rd and v is given) gets
// scale * v[i]; the remaining columns are zero.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_relayout(long n, int ss, int nc, int rd, const T* __restrict__ src, T* __restrict__ dst,
           const double* __restrict__ v, double scale) {
  const long len = n * rd;
  const long stride = (long)gridDim.x * kBlock;
  for (long idx = (long)blockIdx.x * kBlock + threadIdx.x; idx < len; idx += stride) {
    const long i = idx / rd;
    const int c = (int)(idx - i * rd);
    if (c < nc) dst[idx] = src[i * ss + c];
    else if (c == nc && v) dst[idx] = from_acc<T>(static_cast<typename Acc<T>::type>(scale * v[i]));
    else dst[idx] = from_acc<T>(typename Acc<T>::type(0));
  }
}

// Precision conversion (storage), round to nearest even for bfloat16.
template <typename S, typename D>
__global__ void __launch_bounds__(kBlock) k_convert(long len, const S* __restrict__ src, D* __restrict__ dst) {
  const long stride = (long)gridDim.x * kBlock;
  for (long idx = (long)blockIdx.x * kBlock + threadIdx.x; idx < len; idx += stride)
    dst[idx] = from_acc<D>(static_cast<typename Acc<D>::type>(to_acc<S>(src[idx])));
}

// ---- launch helpers ------------------------------------------------------------

void launch_fin_objgrad(const double* part, int nb, DevScalars* sc, double sigma, int mode, double* f_out,
                        hipStream_t st, const BlockTab& tab, int count) {
  hipLaunchKernelGGL(k_fin_objgrad, dim3(count), dim3(kBlock), 0, st, part, nb, sc, sigma, mode, f_out, tab);
}
void launch_fin_step(const double* part_c2, int nb, int c2_stride, DevScalars* sc, double sigma, double j_extra,
                     int mode, double* coeffs_out, double* t_out, hipStream_t st, const BlockTab& tab, int count) {
  hipLaunchKernelGGL(k_fin_step, dim3(count), dim3(kBlock), 0, st, part_c2, nb, c2_stride, sc, sigma, j_extra, mode,
                     coeffs_out, t_out, tab);
}
void launch_fin_ls(const double* part, int nb, DevScalars* sc, double sigma, double* coeffs_out, double* t_out,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_fin_ls, dim3(1), dim3(kBlock), 0, st, part, nb, sc, sigma, coeffs_out, t_out);
}
static int elem_blocks(long len) {
  long nb = (len + kBlock * 4 - 1) / (kBlock * 4);
  if (nb < 1) nb = 1;
  if (nb > 8192) nb = 8192;
  return (int)nb;
}
template <typename T>
void launch_update(long len, T* R, const T* G, const DevScalars* sc, int use_flag, hipStream_t st) {
  hipLaunchKernelGGL((k_update<T>), dim3(elem_blocks(len)), dim3(kBlock), 0, st, len, R, G, sc, use_flag);
}
template void launch_update<double>(long, double*, const double*, const DevScalars*, int, hipStream_t);
template void launch_update<float>(long, float*, const float*, const DevScalars*, int, hipStream_t);
template void launch_update<bf16>(long, bf16*, const bf16*, const DevScalars*, int, hipStream_t);

int dual_blocks(long m) {
  long nb = (m + kBlock * 8 - 1) / (kBlock * 8);
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
  return (int)nb;
}
void launch_dual(long m, const double* Av, const double* b, const double* y_in, double* y_out, double sigma,
                 double* part, DevScalars* sc, double bnorm, double* pinf_out, hipStream_t st, double sigma_tail) {
  const int nb = dual_blocks(m);
  if (!(sigma_tail > 0.0)) sigma_tail = sigma;
  hipLaunchKernelGGL(k_dual, dim3(nb), dim3(kBlock), 0, st, m, Av, b, y_in, y_out, sigma, sigma_tail, part,
                     BlockTab{});
  hipLaunchKernelGGL(k_fin_dual, dim3(1), dim3(kBlock), 0, st, part, nb, sc, bnorm, nullptr, pinf_out, BlockTab{});
}
void launch_dual_batch(long m, const double* Av, const double* b, const double* y_in, double* y_out, double sigma,
                       double* part, DevScalars* sc, const double* bnorms, const BlockTab& tab, int nb, int count,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_dual, dim3(nb), dim3(kBlock), 0, st, m, Av, b, y_in, y_out, sigma, sigma, part, tab);
  hipLaunchKernelGGL(k_fin_dual, dim3(count), dim3(kBlock), 0, st, part, nb, sc, 0.0, bnorms, nullptr, tab);
}
void launch_inner_reset(DevScalars* sc, double tol, int max_inner, int step_rule, double eta, hipStream_t st) {
  hipLaunchKernelGGL(k_inner_reset, dim3(1), dim3(64), 0, st, sc, tol, max_inner, step_rule, eta);
}
void launch_inner_reset_batch(DevScalars* sc, int count, const double* tols, const int32_t* active, int max_inner,
                              int step_rule, double eta, hipStream_t st) {
  hipLaunchKernelGGL(k_inner_reset_batch, dim3((count + 63) / 64), dim3(64), 0, st, sc, count, tols, active,
                     max_inner, step_rule, eta);
}
void launch_copy_active(long m, const double* src, double* dst, const int32_t* active, const BlockTab& tab, int nb,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_copy_active, dim3(nb), dim3(kBlock), 0, st, m, src, dst, active, tab);
}
template <typename T>
void launch_fill_column(long n, int rs, T* R, const double* v, const int32_t* col, const double* scale,
                        const BlockTab& tab, int nb, hipStream_t st) {
  hipLaunchKernelGGL((k_fill_column<T>), dim3(nb), dim3(kBlock), 0, st, n, rs, R, v, col, scale, tab);
}
template void launch_fill_column<double>(long, int, double*, const double*, const int32_t*, const double*,
                                         const BlockTab&, int, hipStream_t);
template void launch_fill_column<float>(long, int, float*, const double*, const int32_t*, const double*,
                                        const BlockTab&, int, hipStream_t);
template void launch_fill_column<bf16>(long, int, bf16*, const double*, const int32_t*, const double*,
                                       const BlockTab&, int, hipStream_t);
template <typename T>
void launch_restride_batch(const BlockTab& tab, int nb, const T* src, T* dst, const int64_t* ob, const int32_t* os,
                           const int64_t* nbase, const int32_t* ns, const int32_t* nc, hipStream_t st) {
  hipLaunchKernelGGL((k_restride_batch<T>), dim3(nb), dim3(kBlock), 0, st, tab, src, dst, ob, os, nbase, ns, nc);
}
template void launch_restride_batch<double>(const BlockTab&, int, const double*, double*, const int64_t*,
                                            const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                                            hipStream_t);
template void launch_restride_batch<float>(const BlockTab&, int, const float*, float*, const int64_t*, const int32_t*,
                                           const int64_t*, const int32_t*, const int32_t*, hipStream_t);
template void launch_restride_batch<bf16>(const BlockTab&, int, const bf16*, bf16*, const int64_t*, const int32_t*,
                                          const int64_t*, const int32_t*, const int32_t*, hipStream_t);

template <typename T>
void launch_set_column(long n, int rs, int c, T* R, const double* v, double scale, hipStream_t st) {
  hipLaunchKernelGGL((k_set_column<T>), dim3(elem_blocks(n)), dim3(kBlock), 0, st, n, rs, c, R, v, scale);
}
template void launch_set_column<double>(long, int, int, double*, const double*, double, hipStream_t);
template void launch_set_column<float>(long, int, int, float*, const double*, double, hipStream_t);
template void launch_set_column<bf16>(long, int, int, bf16*, const double*, double, hipStream_t);

template <typename T>
void launch_relayout(long n, int ss, int nc, int rd, const T* src, T* dst, const double* v, double scale,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_relayout<T>), dim3(elem_blocks(n * rd)), dim3(kBlock), 0, st, n, ss, nc, rd, src, dst, v,
                     scale);
}
template void launch_relayout<double>(long, int, int, int, const double*, double*, const double*, double,
                                      hipStream_t);
template void launch_relayout<float>(long, int, int, int, const float*, float*, const double*, double, hipStream_t);
template void launch_relayout<bf16>(long, int, int, int, const bf16*, bf16*, const double*, double, hipStream_t);

template <typename S, typename D>
void launch_convert(long len, const S* src, D* dst, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<S, D>), dim3(elem_blocks(len)), dim3(kBlock), 0, st, len, src, dst);
}
template void launch_convert<double, float>(long, const double*, float*, hipStream_t);
template void launch_convert<double, bf16>(long, const double*, bf16*, hipStream_t);
template void launch_convert<float, double>(long, const float*, double*, hipStream_t);
template void launch_convert<bf16, double>(long, const bf16*, double*, hipStream_t);
template void launch_convert<bf16, float>(long, const bf16*, float*, hipStream_t);
template void launch_convert<float, bf16>(long, const float*, bf16*, hipStream_t);

}  // namespace almbm
