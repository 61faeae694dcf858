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
               const DevScalars* __restrict__ sc_base, int refresh_every, BlockTab tab, LbfgsRing<RingT<T>> lb) {
  using V = typename Acc<T>::type;
  const Rows ch = rows_of(C.n, tab);
  const DevScalars* sc = sc_base ? sc_base + ch.inst : nullptr;
  if (sc && sc->flag) return;
  // inside the inner loop this full pass runs only on refresh iterations
  if (sc && refresh_every > 1 && (sc->iter % refresh_every) != 0) return;
  // L-BFGS: y_k = G_new - G_old into the current y slot (not on the first step)
  const long xb = row_base(tab, ch.inst);
  RingT<T>* __restrict__ yk =
      (lb.s && sc && sc->iter > 0) ? lb.y + (long)lb.s[ch.inst].cur * lb.stride + xb : nullptr;
  constexpr int RPB = kBlock / LPR;
  const int lane = threadIdx.x % LPR;
  const int slot = threadIdx.x / LPR;
  R += xb;
  if (G) G += xb;
  SplitAcc<NUM_P, LPR> acc;
  acc.zero();
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
    if (yk) {
      V go[VEC], dy[VEC];
      load_frag<T, VEC, FULL>(G + i * r, lane, r, go);
#pragma unroll
      for (int v = 0; v < VEC; ++v) dy[v] = g[v] - go[v];
      store_frag<RingT<T>, VEC, FULL>(yk + i * r, lane, r, dy);
    }
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
    if (lane == 0 && Av) Av[i] = ai;
    {
      const double a1 = 2.0 * (double)rg, a2 = (double)gg;
      acc.add(lane, P_C0, (double)rp);
      acc.add(lane, P_YBMA, yi * (b[i] - ai));
      acc.add(lane, P_EE, ei * ei);
      acc.add(lane, P_GG, a2);
      acc.add(lane, P_GP, (double)gp);
      acc.add(lane, P_YA1, yi * a1);
      acc.add(lane, P_YA2, yi * a2);
      acc.add(lane, P_EA1, ei * a1);
      acc.add(lane, P_EA2, ei * a2);
      acc.add(lane, P_A1A1, a1 * a1);
      acc.add(lane, P_A1A2, a1 * a2);
      acc.add(lane, P_A2A2, a2 * a2);
      acc.add(lane, P_RR, ai);
      acc.add(lane, P_RG, (double)rg);
    }
  }
  acc.block_store(lane, part + part_slot(tab) * NUM_P);
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


// Line-search product of the inner loop: Q = C G stored (arithmetic type) for
// the next step's cost product, and the partial sums of <G, C G>.
template <typename T, int LPR, int VEC, bool FULL>
__global__ void __launch_bounds__(kBlock)
k_quadq_diag(Cost<typename Acc<T>::type> C, int r, const T* __restrict__ G, typename Acc<T>::type* __restrict__ Q,
             double* __restrict__ part, const DevScalars* __restrict__ sc_base, BlockTab tab, LbfgsRing<T> lb) {
  using V = typename Acc<T>::type;
  const Rows ch = rows_of(C.n, tab);
  if (sc_base && sc_base[ch.inst].flag) return;
  if (lb.s) G = lb.e + (long)lb.s[ch.inst].cur * lb.stride;  // L-BFGS: the product of the direction E
  constexpr int RPB = kBlock / LPR;
  const int lane = threadIdx.x % LPR;
  const int slot = threadIdx.x / LPR;
  const long xb = row_base(tab, ch.inst);
  G += xb;
  Q += xb;
  double acc[1] = {0.0};
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V gi[VEC], q[VEC];
    load_frag<T, VEC, FULL>(G + i * r, lane, r, gi);
    spmm_row<T, LPR, VEC, FULL>(C, i, lane, r, G, gi, q);
    store_frag<V, VEC, FULL>(Q + i * r, lane, r, q);
    V gq = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) gq += gi[v] * q[v];
    gq = group_sum<LPR>(gq);
    if (lane == 0) acc[0] += (double)gq;
  }
  block_sum_store<1>(acc, part + part_slot(tab));
}

// Start of an inner iteration: apply the pending step R <- R - t G and, except
// on refresh iterations, evaluate the new gradient without a sparse product.
// The cost product is carried implicitly: before the step P = C R = G/2 + w R
// (w from the stored A(RR^T)), and C (R - t G) = P - t Q with Q = C G from the
// line search, so G_new = 2 (P - t Q - w_new R_new).  Refresh iterations
// (every refresh_every steps) recompute C R with the full sparse pass instead,
// which bounds the drift of the recurrence in reduced precision.
template <typename T, int LPR, int VEC, bool FULL>
__global__ void __launch_bounds__(kBlock)
k_upd_eval_diag(long n, int r, T* __restrict__ R, T* __restrict__ G, const typename Acc<T>::type* __restrict__ Q,
                const double* __restrict__ y, const double* __restrict__ b, double sigma, double* __restrict__ Av,
                double* __restrict__ part, const DevScalars* __restrict__ sc_base, int refresh_every, BlockTab tab,
                LbfgsRing<RingT<T>> lb) {
  using V = typename Acc<T>::type;
  const Rows ch = rows_of(n, tab);
  const DevScalars* sc = sc_base + ch.inst;
  if (sc->flag) return;
  const int e = sc->iter;
  if (e == 0) return;
  // the step is R <- R - t D with D = G (gradient descent) or D = E (L-BFGS,
  // which also writes y_k = G_new - G_old into the current y slot)
  using S = RingT<T>;
  const long xb = row_base(tab, ch.inst);
  const S* __restrict__ D = lb.s ? lb.e + (long)lb.s[ch.inst].cur * lb.stride + xb : nullptr;
  S* __restrict__ yk = lb.s ? lb.y + (long)lb.s[ch.inst].cur * lb.stride + xb : nullptr;
  const bool update_only = refresh_every <= 1 || (e % refresh_every) == 0;
  const V t = static_cast<V>(sc->t);
  constexpr int RPB = kBlock / LPR;
  const int lane = threadIdx.x % LPR;
  const int slot = threadIdx.x / LPR;
  R += xb;
  G += xb;
  Q += xb;
  SplitAcc<NUM_P, LPR> acc;
  acc.zero();
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V ri[VEC], gi[VEC], di[VEC];
    load_frag<T, VEC, FULL>(R + i * r, lane, r, ri);
    load_frag<T, VEC, FULL>(G + i * r, lane, r, gi);
    if (D) load_frag<S, VEC, FULL>(D + i * r, lane, r, di);
    else {
#pragma unroll
      for (int v = 0; v < VEC; ++v) di[v] = gi[v];
    }
    V rn[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) rn[v] = round_st<T>(ri[v] - t * di[v]);
    store_frag<T, VEC, FULL>(R + i * r, lane, r, rn);
    if (update_only) continue;
    V qi[VEC];
    load_frag<V, VEC, FULL>(Q + i * r, lane, r, qi);
    const double yi = y[i], bi = b[i];
    const V w_old = static_cast<V>(yi - sigma * (Av[i] - bi));
    V p[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) p[v] = V(0.5) * gi[v] + w_old * ri[v] - t * qi[v];
    V rr = 0, rp = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      rr += rn[v] * rn[v];
      rp += rn[v] * p[v];
    }
    rr = group_sum<LPR>(rr);
    rp = group_sum<LPR>(rp);
    const double ai = rr;
    const double ei = ai - bi;
    const V wv = static_cast<V>(yi - sigma * ei);
    V g[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) g[v] = round_st<T>(V(2) * (p[v] - wv * rn[v]));
    if (yk) {
      V dy[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) dy[v] = g[v] - gi[v];
      store_frag<S, VEC, FULL>(yk + i * r, lane, r, dy);
    }
    store_frag<T, VEC, FULL>(G + i * r, lane, r, g);
    V gg = 0, gp = 0, rg = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      gg += g[v] * g[v];
      gp += g[v] * p[v];
      rg += rn[v] * g[v];
    }
    gg = group_sum<LPR>(gg);
    gp = group_sum<LPR>(gp);
    rg = group_sum<LPR>(rg);
    if (lane == 0) Av[i] = ai;
    {
      const double a1 = 2.0 * (double)rg, a2 = (double)gg;
      acc.add(lane, P_C0, (double)rp);
      acc.add(lane, P_YBMA, yi * (bi - ai));
      acc.add(lane, P_EE, ei * ei);
      acc.add(lane, P_GG, a2);
      acc.add(lane, P_GP, (double)gp);
      acc.add(lane, P_YA1, yi * a1);
      acc.add(lane, P_YA2, yi * a2);
      acc.add(lane, P_EA1, ei * a1);
      acc.add(lane, P_EA2, ei * a2);
      acc.add(lane, P_A1A1, a1 * a1);
      acc.add(lane, P_A1A2, a1 * a2);
      acc.add(lane, P_A2A2, a2 * a2);
      acc.add(lane, P_RR, ai);
      acc.add(lane, P_RG, (double)rg);
    }
  }
  if (!update_only) acc.block_store(lane, part + part_slot(tab) * NUM_P);
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
  SplitAcc<NUM_P, LPR> acc;
  acc.zero();
  Cost<V> CG = C;  // the product C G reads its hub sums from hsum2
  CG.hsum = C.hsum2;
  const RowChunk ch = row_chunk(C.n);
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V ri[VEC], gi[VEC], p[VEC], q[VEC];
    load_frag<T, VEC, FULL>(R + i * r, lane, r, ri);
    load_frag<T, VEC, FULL>(G + i * r, lane, r, gi);
    spmm_row<T, LPR, VEC, FULL>(C, i, lane, r, R, ri, p);
    spmm_row<T, LPR, VEC, FULL>(CG, i, lane, r, G, gi, q);
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
    {
      const double ai = rr, yi = y[i], ei = ai - b[i];
      const double a1 = 2.0 * (double)rg, a2 = (double)gg;
      acc.add(lane, P_C0, (double)rp);
      acc.add(lane, P_YBMA, yi * (b[i] - ai));
      acc.add(lane, P_EE, ei * ei);
      acc.add(lane, P_GG, a2);
      acc.add(lane, P_GP, (double)gp);
      acc.add(lane, P_YA1, yi * a1);
      acc.add(lane, P_YA2, yi * a2);
      acc.add(lane, P_EA1, ei * a1);
      acc.add(lane, P_EA2, ei * a2);
      acc.add(lane, P_A1A1, a1 * a1);
      acc.add(lane, P_A1A2, a1 * a2);
      acc.add(lane, P_A2A2, a2 * a2);
      acc.add(lane, P_RR, ai);
      acc.add(lane, P_RG, (double)rg);
      acc.add(lane, P_C2, (double)gq);
    }
  }
  acc.block_store(lane, part + (long)blockIdx.x * NUM_P);
}

// ---- launchers -----------------------------------------------------------------

// Neighbour sums of the hub rows (see Cost): out[h, :] = sum_k S_ik X_k for
// i = hrow[h], without the diagonal term.  One block per hub: its kBlock/LPR
// lane groups take every (kBlock/LPR)-th entry of the row with kUnroll gathers
// in flight each, and the groups' sums are added in group order, so the result
// does not depend on timing.  The same early exits as the row kernel that
// consumes the sums (converged flag, non-refresh iterations).
template <typename T, int LPR, int VEC, bool FULL>
__global__ void __launch_bounds__(kBlock)
k_hub_rows(Cost<typename Acc<T>::type> C, int r, const T* __restrict__ X, typename Acc<T>::type* __restrict__ out,
           const DevScalars* __restrict__ sc, int refresh_every, LbfgsRing<T> lb) {
  using V = typename Acc<T>::type;
  if (sc && sc->flag) return;
  if (sc && refresh_every > 1 && (sc->iter % refresh_every) != 0) return;
  if (lb.s) X = lb.e + (long)lb.s->cur * lb.stride;  // L-BFGS line-search product: the direction E
  constexpr int NG = kBlock / LPR;
  constexpr int U = kUnroll;
  const int lane = threadIdx.x % LPR;
  const int grp = threadIdx.x / LPR;
  __shared__ V buf[NG][LPR * VEC];
  for (long h = blockIdx.x; h < C.nh; h += gridDim.x) {
    const long i = C.hrow[h];
    const long k0 = C.rp[i], k1 = C.rp[i + 1];
    V p[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) p[v] = V(0);
    for (long k = k0 + grp; k < k1; k += (long)NG * U) {
      V x[U][VEC];
      V c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long kk = k + (long)u * NG;
        const bool in = kk < k1;
        const int j = in ? C.ci[kk] : (int)i;
        c[u] = in ? C.cv[kk] : V(0);
        load_frag<T, VEC, FULL>(X + (long)j * r, lane, r, x[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < VEC; ++v) p[v] += c[u] * x[u][v];
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) buf[grp][lane * VEC + v] = p[v];
    __syncthreads();
    for (int c = threadIdx.x; c < r; c += kBlock) {
      V s = V(0);
      for (int g = 0; g < NG; ++g) s += buf[g][c];
      out[h * r + c] = s;
    }
    __syncthreads();
  }
}

template <typename T, int LPR, int VEC>
static void launch_hub_cfg(const Cost<typename Acc<T>::type>& C, int r, const T* X, typename Acc<T>::type* out,
                           const DevScalars* sc, int refresh_every, hipStream_t st, const LbfgsRing<T>& lb) {
  const int nb = C.nh < 65536 ? C.nh : 65536;
  if (r == LPR * VEC)
    hipLaunchKernelGGL((k_hub_rows<T, LPR, VEC, true>), dim3(nb), dim3(kBlock), 0, st, C, r, X, out, sc,
                       refresh_every, lb);
  else
    hipLaunchKernelGGL((k_hub_rows<T, LPR, VEC, false>), dim3(nb), dim3(kBlock), 0, st, C, r, X, out, sc,
                       refresh_every, lb);
}

template <typename T, int LPR, int VEC>
static void launch_objgrad_cfg(const Cost<typename Acc<T>::type>& C, int r, const T* R, const double* y,
                               const double* b, double sigma, T* G, double* Av, double* part,
                               const DevScalars* sc, int refresh_every, const BlockTab& tab, int nblk,
                               hipStream_t st, const LbfgsRing<RingT<T>>& lb) {
  if (r == LPR * VEC)
    hipLaunchKernelGGL((k_objgrad_diag<T, LPR, VEC, true>), dim3(nblk), dim3(kBlock), 0, st, C, r, R, y, b,
                       sigma, G, Av, part, sc, refresh_every, tab, lb);
  else
    hipLaunchKernelGGL((k_objgrad_diag<T, LPR, VEC, false>), dim3(nblk), dim3(kBlock), 0, st, C, r, R, y, b,
                       sigma, G, Av, part, sc, refresh_every, tab, lb);
}

template <typename T, int LPR, int VEC>
static void launch_quadq_cfg(const Cost<typename Acc<T>::type>& C, int r, const T* G, typename Acc<T>::type* Q,
                             double* part, const DevScalars* sc, const BlockTab& tab, int nblk, hipStream_t st,
                             const LbfgsRing<T>& lb) {
  if (r == LPR * VEC)
    hipLaunchKernelGGL((k_quadq_diag<T, LPR, VEC, true>), dim3(nblk), dim3(kBlock), 0, st, C, r, G, Q, part, sc, tab,
                       lb);
  else
    hipLaunchKernelGGL((k_quadq_diag<T, LPR, VEC, false>), dim3(nblk), dim3(kBlock), 0, st, C, r, G, Q, part, sc,
                       tab, lb);
}

template <typename T, int LPR, int VEC>
static void launch_upd_eval_cfg(long n, int r, T* R, T* G, const typename Acc<T>::type* Q, const double* y,
                                const double* b, double sigma, double* Av, double* part, const DevScalars* sc,
                                int refresh_every, const BlockTab& tab, int nblk, hipStream_t st,
                                const LbfgsRing<RingT<T>>& lb) {
  if (r == LPR * VEC)
    hipLaunchKernelGGL((k_upd_eval_diag<T, LPR, VEC, true>), dim3(nblk), dim3(kBlock), 0, st, n, r, R, G, Q, y, b,
                       sigma, Av, part, sc, refresh_every, tab, lb);
  else
    hipLaunchKernelGGL((k_upd_eval_diag<T, LPR, VEC, false>), dim3(nblk), dim3(kBlock), 0, st, n, r, R, G, Q, y, b,
                       sigma, Av, part, sc, refresh_every, tab, lb);
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


template <typename T>
void launch_hub_rows(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* X,
                     typename Acc<T>::type* out, const DevScalars* sc, int refresh_every, hipStream_t st,
                     const LbfgsRing<T>& lb) {
  if (C.nh <= 0) return;
  ALMBM_DISPATCH_DIAG(T, launch_hub_cfg, C, r, X, out, sc, refresh_every, st, lb);
}

template <typename T>
void launch_objgrad_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* R, const double* y,
                         const double* b, double sigma, T* G, double* Av, double* part, const DevScalars* sc,
                         int refresh_every, const BlockTab& tab, int nblk, hipStream_t st,
                         const LbfgsRing<RingT<T>>& lb) {
  launch_hub_rows<T>(C, r, variant, R, C.hsum, sc, refresh_every, st, LbfgsRing<T>{});
  ALMBM_DISPATCH_DIAG(T, launch_objgrad_cfg, C, r, R, y, b, sigma, G, Av, part, sc, refresh_every, tab, nblk, st,
                      lb);
}

template <typename T>
void launch_quadq_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* G,
                       typename Acc<T>::type* Q, double* part, const DevScalars* sc, const BlockTab& tab, int nblk,
                       hipStream_t st, const LbfgsRing<T>& lb) {
  launch_hub_rows<T>(C, r, variant, G, C.hsum, sc, 0, st, lb);
  ALMBM_DISPATCH_DIAG(T, launch_quadq_cfg, C, r, G, Q, part, sc, tab, nblk, st, lb);
}

template <typename T>
void launch_upd_eval_diag(long n, int r, int variant, T* R, T* G, const typename Acc<T>::type* Q, const double* y,
                          const double* b, double sigma, double* Av, double* part, const DevScalars* sc,
                          int refresh_every, const BlockTab& tab, int nblk, hipStream_t st,
                          const LbfgsRing<RingT<T>>& lb) {
  ALMBM_DISPATCH_DIAG(T, launch_upd_eval_cfg, n, r, R, G, Q, y, b, sigma, Av, part, sc, refresh_every, tab, nblk, st,
                      lb);
}

template <typename T>
void launch_quad_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* G, double* part,
                      const DevScalars* sc, int nblk, hipStream_t st) {
  launch_hub_rows<T>(C, r, variant, G, C.hsum, sc, 0, st, LbfgsRing<T>{});
  ALMBM_DISPATCH_DIAG(T, launch_quad_cfg, C, r, G, part, sc, nblk, st);
}

template <typename T>
void launch_ls_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* R, const T* G,
                    const double* y, const double* b, double* part, int nblk, hipStream_t st) {
  launch_hub_rows<T>(C, r, variant, R, C.hsum, nullptr, 0, st, LbfgsRing<T>{});
  launch_hub_rows<T>(C, r, variant, G, C.hsum2, nullptr, 0, st, LbfgsRing<T>{});
  ALMBM_DISPATCH_DIAG(T, launch_ls_cfg, C, r, R, G, y, b, part, nblk, st);
}

#define ALMBM_INST(T)                                                                                     \
  template void launch_objgrad_diag<T>(const Cost<Acc<T>::type>&, int, int, const T*, const double*,      \
                                       const double*, double, T*, double*, double*, const DevScalars*, int, \
                                       const BlockTab&, int, hipStream_t, const LbfgsRing<RingT<T>>&);    \
  template void launch_quadq_diag<T>(const Cost<Acc<T>::type>&, int, int, const T*, Acc<T>::type*, double*, \
                                     const DevScalars*, const BlockTab&, int, hipStream_t,                 \
                                     const LbfgsRing<T>&);                                                 \
  template void launch_upd_eval_diag<T>(long, int, int, T*, T*, const Acc<T>::type*, const double*,          \
                                        const double*, double, double*, double*, const DevScalars*, int,     \
                                        const BlockTab&, int, hipStream_t, const LbfgsRing<RingT<T>>&);     \
  template void launch_quad_diag<T>(const Cost<Acc<T>::type>&, int, int, const T*, double*,               \
                                    const DevScalars*, int, hipStream_t);                                 \
  template void launch_ls_diag<T>(const Cost<Acc<T>::type>&, int, int, const T*, const T*, const double*,  \
                                  const double*, double*, int, hipStream_t);                              \
  template void launch_hub_rows<T>(const Cost<Acc<T>::type>&, int, int, const T*, Acc<T>::type*,          \
                                   const DevScalars*, int, hipStream_t, const LbfgsRing<T>&);

ALMBM_INST(double)
ALMBM_INST(float)
ALMBM_INST(bf16)

}  // namespace almbm
