// Row kernels for the DIAG constraint family (A_i = e_i e_i^T, m = n): the
// MaxCut relaxation of Sec. 6.1 and any cost C = S + Diag(d).
//
// One row group of LPR lanes owns a row i of R; lane l keeps columns
// [l*VEC, l*VEC+VEC) in registers.  The sparse product (CR)_i = d_i R_i +
// sum_k S_ik R_k gathers whole rows of R (one coalesced LPR-lane access each),
// then the epilogue forms a_i = ||R_i||^2, w_i = y_i - sigma (a_i - b_i) and
// G_i = 2 (P_i - w_i R_i) (the gradient 2 (C - A*(w)) R of eq. AL-BM) and the
// per-row terms of the objective and of the quartic line search.  No MFMA: the
// work is a sparse gather at ~2r flop per 12 B of matrix plus r*sizeof(T) of
// gathered row, far below the vector ALU balance, so the kernels are bound by
// HBM/Infinity-Cache bandwidth.
#include "spmm_row.hpp"

namespace almbm {

// Fused objective + gradient + line-search partials (the hot kernel).
template <typename T, int LPR, int VEC, bool FULL>
__global__ void __launch_bounds__(kBlock)
k_objgrad_diag(Cost<typename Acc<T>::type> C, int r, const T* __restrict__ R,
               const double* __restrict__ y, const double* __restrict__ b, double sigma,
               T* __restrict__ G, double* __restrict__ Av, double* __restrict__ part,
               const DevScalars* __restrict__ sc) {
  using V = typename Acc<T>::type;
  if (sc && sc->flag) return;
  constexpr int RPB = kBlock / LPR;
  const int lane = threadIdx.x % LPR;
  const int slot = threadIdx.x / LPR;
  double acc[NUM_P];
#pragma unroll
  for (int s = 0; s < NUM_P; ++s) acc[s] = 0.0;
  const RowChunk ch = row_chunk(C.n);
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V ri[VEC], p[VEC];
    load_frag<T, VEC, FULL>(R + i * r, lane, r, ri);
    spmm_row<T, LPR, VEC, FULL>(C, i, lane, r, R, ri, p);
    V rr = 0, rp = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      rr += ri[v] * ri[v];
      rp += ri[v] * p[v];
    }
    rr = group_sum<LPR>(rr);
    rp = group_sum<LPR>(rp);
    const double ai = rr;
    const double yi = y[i];
    const double ei = ai - b[i];
    const double wi = yi - sigma * ei;
    const V wv = static_cast<V>(wi);
    V g[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) g[v] = round_st<T>(V(2) * (p[v] - wv * ri[v]));
    if (G) store_frag<T, VEC, FULL>(G + i * r, lane, r, g);
    V gg = 0, gp = 0, rg = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      gg += g[v] * g[v];
      gp += g[v] * p[v];
      rg += ri[v] * g[v];
    }
    gg = group_sum<LPR>(gg);
    gp = group_sum<LPR>(gp);
    rg = group_sum<LPR>(rg);
    if (lane == 0) {
      if (Av) Av[i] = ai;
      const double a1 = 2.0 * (double)rg, a2 = (double)gg;
      acc[P_C0] += (double)rp;
      acc[P_YBMA] += yi * (b[i] - ai);
      acc[P_EE] += ei * ei;
      acc[P_GG] += a2;
      acc[P_GP] += (double)gp;
      acc[P_YA1] += yi * a1;
      acc[P_YA2] += yi * a2;
      acc[P_EA1] += ei * a1;
      acc[P_EA2] += ei * a2;
      acc[P_A1A1] += a1 * a1;
      acc[P_A1A2] += a1 * a2;
      acc[P_A2A2] += a2 * a2;
      acc[P_RR] += ai;
      acc[P_RG] += (double)rg;
    }
  }
  block_sum_store<NUM_P>(acc, part + (long)blockIdx.x * NUM_P);
}

// c2 = <G, C G> for the quartic line search (sparse product of the direction).
template <typename T, int LPR, int VEC, bool FULL>
__global__ void __launch_bounds__(kBlock)
k_quad_diag(Cost<typename Acc<T>::type> C, int r, const T* __restrict__ G,
            double* __restrict__ part, const DevScalars* __restrict__ sc) {
  using V = typename Acc<T>::type;
  if (sc && sc->flag) return;
  constexpr int RPB = kBlock / LPR;
  const int lane = threadIdx.x % LPR;
  const int slot = threadIdx.x / LPR;
  double acc[1] = {0.0};
  const RowChunk ch = row_chunk(C.n);
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V gi[VEC], q[VEC];
    load_frag<T, VEC, FULL>(G + i * r, lane, r, gi);
    spmm_row<T, LPR, VEC, FULL>(C, i, lane, r, G, gi, q);
    V gq = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) gq += gi[v] * q[v];
    gq = group_sum<LPR>(gq);
    if (lane == 0) acc[0] += (double)gq;
  }
  block_sum_store<1>(acc, part + blockIdx.x);
}

// All line-search partials for an arbitrary direction G (API entry point).
template <typename T, int LPR, int VEC, bool FULL>
__global__ void __launch_bounds__(kBlock)
k_ls_diag(Cost<typename Acc<T>::type> C, int r, const T* __restrict__ R, const T* __restrict__ G,
          const double* __restrict__ y, const double* __restrict__ b,
          double* __restrict__ part) {
  using V = typename Acc<T>::type;
  constexpr int RPB = kBlock / LPR;
  const int lane = threadIdx.x % LPR;
  const int slot = threadIdx.x / LPR;
  double acc[NUM_P];
#pragma unroll
  for (int s = 0; s < NUM_P; ++s) acc[s] = 0.0;
  const RowChunk ch = row_chunk(C.n);
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V ri[VEC], gi[VEC], p[VEC], q[VEC];
    load_frag<T, VEC, FULL>(R + i * r, lane, r, ri);
    load_frag<T, VEC, FULL>(G + i * r, lane, r, gi);
    spmm_row<T, LPR, VEC, FULL>(C, i, lane, r, R, ri, p);
    spmm_row<T, LPR, VEC, FULL>(C, i, lane, r, G, gi, q);
    V rr = 0, rp = 0, gg = 0, gp = 0, rg = 0, gq = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      rr += ri[v] * ri[v];
      rp += ri[v] * p[v];
      gg += gi[v] * gi[v];
      gp += gi[v] * p[v];
      rg += ri[v] * gi[v];
      gq += gi[v] * q[v];
    }
    rr = group_sum<LPR>(rr);
    rp = group_sum<LPR>(rp);
    gg = group_sum<LPR>(gg);
    gp = group_sum<LPR>(gp);
    rg = group_sum<LPR>(rg);
    gq = group_sum<LPR>(gq);
    if (lane == 0) {
      const double ai = rr, yi = y[i], ei = ai - b[i];
      const double a1 = 2.0 * (double)rg, a2 = (double)gg;
      acc[P_C0] += (double)rp;
      acc[P_YBMA] += yi * (b[i] - ai);
      acc[P_EE] += ei * ei;
      acc[P_GG] += a2;
      acc[P_GP] += (double)gp;
      acc[P_YA1] += yi * a1;
      acc[P_YA2] += yi * a2;
      acc[P_EA1] += ei * a1;
      acc[P_EA2] += ei * a2;
      acc[P_A1A1] += a1 * a1;
      acc[P_A1A2] += a1 * a2;
      acc[P_A2A2] += a2 * a2;
      acc[P_RR] += ai;
      acc[P_RG] += (double)rg;
      acc[P_C2] += (double)gq;
    }
  }
  block_sum_store<NUM_P>(acc, part + (long)blockIdx.x * NUM_P);
}

// ---- launchers -----------------------------------------------------------------

template <typename T, int LPR, int VEC>
static void launch_objgrad_cfg(const Cost<typename Acc<T>::type>& C, int r, const T* R, const double* y,
                               const double* b, double sigma, T* G, double* Av, double* part,
                               const DevScalars* sc, int nblk, hipStream_t st) {
  if (r == LPR * VEC)
    hipLaunchKernelGGL((k_objgrad_diag<T, LPR, VEC, true>), dim3(nblk), dim3(kBlock), 0, st, C, r, R, y, b,
                       sigma, G, Av, part, sc);
  else
    hipLaunchKernelGGL((k_objgrad_diag<T, LPR, VEC, false>), dim3(nblk), dim3(kBlock), 0, st, C, r, R, y, b,
                       sigma, G, Av, part, sc);
}

template <typename T, int LPR, int VEC>
static void launch_quad_cfg(const Cost<typename Acc<T>::type>& C, int r, const T* G, double* part,
                            const DevScalars* sc, int nblk, hipStream_t st) {
  if (r == LPR * VEC)
    hipLaunchKernelGGL((k_quad_diag<T, LPR, VEC, true>), dim3(nblk), dim3(kBlock), 0, st, C, r, G, part, sc);
  else
    hipLaunchKernelGGL((k_quad_diag<T, LPR, VEC, false>), dim3(nblk), dim3(kBlock), 0, st, C, r, G, part, sc);
}

template <typename T, int LPR, int VEC>
static void launch_ls_cfg(const Cost<typename Acc<T>::type>& C, int r, const T* R, const T* G, const double* y,
                          const double* b, double* part, int nblk, hipStream_t st) {
  if (r == LPR * VEC)
    hipLaunchKernelGGL((k_ls_diag<T, LPR, VEC, true>), dim3(nblk), dim3(kBlock), 0, st, C, r, R, G, y, b, part);
  else
    hipLaunchKernelGGL((k_ls_diag<T, LPR, VEC, false>), dim3(nblk), dim3(kBlock), 0, st, C, r, R, G, y, b, part);
}

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

template <typename T>
void launch_objgrad_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* R, const double* y,
                         const double* b, double sigma, T* G, double* Av, double* part, const DevScalars* sc,
                         int nblk, hipStream_t st) {
  ALMBM_DISPATCH_DIAG(T, launch_objgrad_cfg, C, r, R, y, b, sigma, G, Av, part, sc, nblk, st);
}

template <typename T>
void launch_quad_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* G, double* part,
                      const DevScalars* sc, int nblk, hipStream_t st) {
  ALMBM_DISPATCH_DIAG(T, launch_quad_cfg, C, r, G, part, sc, nblk, st);
}

template <typename T>
void launch_ls_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* R, const T* G,
                    const double* y, const double* b, double* part, int nblk, hipStream_t st) {
  ALMBM_DISPATCH_DIAG(T, launch_ls_cfg, C, r, R, G, y, b, part, nblk, st);
}

#define ALMBM_INST(T)                                                                                     \
  template void launch_objgrad_diag<T>(const Cost<Acc<T>::type>&, int, int, const T*, const double*,      \
                                       const double*, double, T*, double*, double*, const DevScalars*, int, \
                                       hipStream_t);                                                      \
  template void launch_quad_diag<T>(const Cost<Acc<T>::type>&, int, int, const T*, double*,               \
                                    const DevScalars*, int, hipStream_t);                                 \
  template void launch_ls_diag<T>(const Cost<Acc<T>::type>&, int, int, const T*, const T*, const double*,  \
                                  const double*, double*, int, hipStream_t);

ALMBM_INST(double)
ALMBM_INST(float)
ALMBM_INST(bf16)

}  // namespace almbm
