// L-BFGS subproblem solver of the inner loop (DIAG family): the direction
// E = H G of the limited-memory BFGS inverse-Hessian estimate built from the
// last m pairs (s, y), taken with the same exact quartic line search as
// gradient descent (R <- R - t E).  SDPLR, the ALM-BM solver Sec. 2 names,
// solves its subproblems this way.
//
// Per step, after the gradient pass (which also writes y_k = G_new - G_old):
//   k_lbfgs_dots      inner products of G and y_k with the stored vectors
//   k_fin_lbfgs       takes the pair (s_k, y_k) if s_k^T y_k > 0 (relative
//                     to ||s|| ||y||), updates the small Gram matrices and
//                     runs the two-loop recursion on coefficients
//   k_lbfgs_combine   E = cg G + sum_a (ce_a E_a + cy_a y_a) and the
//                     quartic's direction-dependent partial sums
//   k_fin_lsdir       their totals
// then the line-search product C E and the step rule as for gradient descent.
// Pure streaming kernels: no gathers, no MFMA.
#include "spmm_row.hpp"

namespace almbm {

// ---- reset -----------------------------------------------------------------------

// One block per instance (state s + blockIdx.x).
__global__ void k_lbfgs_reset(LbfgsState* s, int m) {
  if (threadIdx.x != 0) return;
  s += blockIdx.x;
  s->m = m;
  s->cnt = 0;
  s->cur = 0;
  s->have = 0;
  s->resets = 0;
  s->accepted = 0;
  s->ee = 0.0;
  s->cg = 1.0;
  for (int a = 0; a < kMaxLbfgs; ++a) {
    s->ord[a] = 0;
    s->ce[a] = 0.0;
    s->cy[a] = 0.0;
  }
  for (int a = 0; a < kLbfgsSlots; ++a) s->tp[a] = 0.0;
}

// ---- inner products ------------------------------------------------------------
//
// Partial slots per block, kLbfgsSlots each: G . E_a, G . y_a, y_k . E_a,
// y_k . y_a for the held pairs a < cnt in set order at positions a and for the
// current direction (E_k, y_k) at position kMaxLbfgs; then E_k . y_a (a < cnt).
// The y_k and E_k products only when a direction was taken (have).

template <typename T> struct FlatVec { static constexpr int N = 16 / sizeof(T); };

template <typename T, int N>
__device__ __forceinline__ void load_flat(const T* __restrict__ p, typename Acc<T>::type (&out)[N]) {
  if constexpr (N == 1) {
    out[0] = to_acc<T>(p[0]);
  } else {
    using W = typename VecWord<N * sizeof(T)>::type;
    W w = *reinterpret_cast<const W*>(p);
    const T* e = reinterpret_cast<const T*>(&w);
#pragma unroll
    for (int v = 0; v < N; ++v) out[v] = to_acc<T>(e[v]);
  }
}

template <typename V> struct DotAcc {
  V gE[kLbfgsSlots], gY[kLbfgsSlots], kE[kLbfgsSlots], kY[kLbfgsSlots], eY[kMaxLbfgs];
};

// NV consecutive elements at idx of every vector.
template <typename T, int NV, typename S = RingT<T>>
__device__ __forceinline__ void dots_chunk(DotAcc<typename Acc<T>::type>& A, long idx, const T* __restrict__ G,
                                           const S* __restrict__ yk, const S* __restrict__ ek,
                                           const S* const (&ea)[kMaxLbfgs], const S* const (&ya)[kMaxLbfgs],
                                           int cnt, bool have) {
  using V = typename Acc<T>::type;
  V g[NV], y_k[NV], e_k[NV];
  load_flat<T, NV>(G + idx, g);
  if (have) {
    load_flat<S, NV>(yk + idx, y_k);
    load_flat<S, NV>(ek + idx, e_k);
  }
#pragma unroll
  for (int a = 0; a < kMaxLbfgs; ++a) {
    if (a < cnt) {
      V ev[NV], yv[NV];
      load_flat<S, NV>(ea[a] + idx, ev);
      load_flat<S, NV>(ya[a] + idx, yv);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        A.gE[a] += g[v] * ev[v];
        A.gY[a] += g[v] * yv[v];
      }
      if (have) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          A.kE[a] += y_k[v] * ev[v];
          A.kY[a] += y_k[v] * yv[v];
          A.eY[a] += e_k[v] * yv[v];
        }
      }
    }
  }
  if (have) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      A.gE[kMaxLbfgs] += g[v] * e_k[v];
      A.gY[kMaxLbfgs] += g[v] * y_k[v];
      A.kE[kMaxLbfgs] += y_k[v] * e_k[v];
      A.kY[kMaxLbfgs] += y_k[v] * y_k[v];
    }
  }
}

// Without a table the grid strides over all len elements.  With a table each
// block takes the elements of its rows, [xbase + lo r, xbase + hi r) of its
// instance (stored at width r), with the instance's own state and stop flag.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_lbfgs_dots(long len, int r, const T* __restrict__ G, LbfgsRing<RingT<T>> lb, double* __restrict__ part,
             const DevScalars* __restrict__ sc_base, BlockTab tab) {
  using V = typename Acc<T>::type;
  using R = RingT<T>;
  constexpr int N = FlatVec<T>::N;
  long a = 0, e = len, t0 = (long)blockIdx.x * kBlock + threadIdx.x, tstride = (long)gridDim.x * kBlock;
  int inst = 0;
  if (tab.inst) {
    inst = tab.inst[blockIdx.x];
    const long xb = row_base(tab, inst);
    a = xb + (long)tab.lo[blockIdx.x] * r;
    e = xb + (long)tab.hi[blockIdx.x] * r;
    t0 = threadIdx.x;
    tstride = kBlock;
  }
  if (sc_base[inst].flag) return;
  const LbfgsState* S = lb.s + inst;
  const int cnt = S->cnt;
  const bool have = S->have != 0;
  const R* yk = lb.y + (long)S->cur * lb.stride;
  const R* ek = lb.e + (long)S->cur * lb.stride;
  const R* ea[kMaxLbfgs];
  const R* ya[kMaxLbfgs];
#pragma unroll
  for (int a = 0; a < kMaxLbfgs; ++a) {
    const int sl = a < cnt ? S->ord[a] : 0;
    ea[a] = lb.e + (long)sl * lb.stride;
    ya[a] = lb.y + (long)sl * lb.stride;
  }
  DotAcc<V> A;
#pragma unroll
  for (int a = 0; a < kLbfgsSlots; ++a) A.gE[a] = A.gY[a] = A.kE[a] = A.kY[a] = V(0);
#pragma unroll
  for (int a = 0; a < kMaxLbfgs; ++a) A.eY[a] = V(0);
  // element-wise head up to N-element alignment, N-element chunks, element-wise tail
  const long pad = (N - a % N) % N;
  const long a_al = a + pad < e ? a + pad : e;
  for (long idx = a + t0; idx < a_al; idx += tstride) dots_chunk<T, 1>(A, idx, G, yk, ek, ea, ya, cnt, have);
  const long nvec = (e - a_al) / N;
  for (long q = t0; q < nvec; q += tstride) dots_chunk<T, N>(A, a_al + q * N, G, yk, ek, ea, ya, cnt, have);
  for (long idx = a_al + nvec * N + t0; idx < e; idx += tstride)
    dots_chunk<T, 1>(A, idx, G, yk, ek, ea, ya, cnt, have);
  double acc[kLbfgsDots];
#pragma unroll
  for (int a = 0; a < kLbfgsSlots; ++a) {
    acc[a] = (double)A.gE[a];
    acc[kLbfgsSlots + a] = (double)A.gY[a];
    acc[2 * kLbfgsSlots + a] = (double)A.kE[a];
    acc[3 * kLbfgsSlots + a] = (double)A.kY[a];
    acc[4 * kLbfgsSlots + a] = a < kMaxLbfgs ? (double)A.eY[a] : 0.0;
  }
  block_sum_store<kLbfgsDots>(acc, part + part_slot(tab) * kLbfgsDots);
}

// ---- pair update and the two-loop recursion on coefficients ----------------------

// One block per instance (blockIdx.x; a single instance without a table).
__global__ void __launch_bounds__(kBlock)
k_fin_lbfgs(const double* __restrict__ part, int nb, const DevScalars* __restrict__ sc_base,
            LbfgsState* __restrict__ S_base, BlockTab tab) {
  const DevScalars* sc = sc_base + blockIdx.x;
  LbfgsState* S = S_base + blockIdx.x;
  if (sc->flag) return;
  int b0, b1;
  inst_blocks(tab, blockIdx.x, nb, b0, b1);
  // fixed-order totals: thread t sums blocks b0 + t, b0 + t + kBlock, ..., then the block tree
  double acc[kLbfgsDots];
#pragma unroll
  for (int k = 0; k < kLbfgsDots; ++k) acc[k] = 0.0;
  for (int bi = b0 + threadIdx.x; bi < b1; bi += kBlock)
#pragma unroll
    for (int k = 0; k < kLbfgsDots; ++k) acc[k] += part[(long)bi * kLbfgsDots + k];
  __shared__ double tot[kLbfgsDots];
  block_sum_store<kLbfgsDots>(acc, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double* gE = tot;
  const double* gY = tot + kLbfgsSlots;
  const double* kE = tot + 2 * kLbfgsSlots;
  const double* kY = tot + 3 * kLbfgsSlots;
  const double* eY = tot + 4 * kLbfgsSlots;
  const int m = S->m;
  int c = S->cnt;
  const int cur = S->cur;
  const double t = sc->t;  // the step just taken along E_k
  // products of G with the held pairs, in set order after the update below
  double gsE[kMaxLbfgs], gsY[kMaxLbfgs];
  for (int a = 0; a < c; ++a) {
    gsE[a] = gE[a];
    gsY[a] = gY[a];
  }
  int next = cur;
  if (S->have) {
    if (!(t > 0.0)) {
      // a zero step: clear the memory, the next direction is the gradient
      c = 0;
      S->resets += 1;
    } else {
      const double sy = -t * kE[kMaxLbfgs];  // s_k . y_k with s_k = -t E_k
      const double ss = t * t * S->ee;
      const double yy = kY[kMaxLbfgs];
      if (sy > 1e-12 * sqrt(ss) * sqrt(yy)) {
        double col[kMaxLbfgs], row[kMaxLbfgs], yrow[kMaxLbfgs];
        for (int a = 0; a < c; ++a) {
          col[a] = -S->tp[S->ord[a]] * kE[a];  // s_a . y_k
          row[a] = -t * eY[a];                 // s_k . y_a
          yrow[a] = kY[a];                     // y_k . y_a
        }
        const double gE_new = gE[kMaxLbfgs], gY_new = gY[kMaxLbfgs];
        if (c == m) {  // drop the oldest pair
          next = S->ord[0];
          for (int a = 0; a + 1 < c; ++a) {
            S->ord[a] = S->ord[a + 1];
            gsE[a] = gsE[a + 1];
            gsY[a] = gsY[a + 1];
            col[a] = col[a + 1];
            row[a] = row[a + 1];
            yrow[a] = yrow[a + 1];
            for (int b = 0; b + 1 < c; ++b) {
              S->SY[a][b] = S->SY[a + 1][b + 1];
              S->YY[a][b] = S->YY[a + 1][b + 1];
            }
          }
          c -= 1;
        } else {
          // first slot held by no pair and not the current one
          for (int sl = 0; sl < kLbfgsSlots; ++sl) {
            bool used = sl == cur;
            for (int a = 0; a < c; ++a) used = used || S->ord[a] == sl;
            if (!used) {
              next = sl;
              break;
            }
          }
        }
        S->tp[cur] = t;
        S->ord[c] = cur;
        for (int a = 0; a < c; ++a) {
          S->SY[a][c] = col[a];
          S->SY[c][a] = row[a];
          S->YY[a][c] = S->YY[c][a] = yrow[a];
        }
        S->SY[c][c] = sy;
        S->YY[c][c] = yy;
        gsE[c] = gE_new;
        gsY[c] = gY_new;
        c += 1;
        S->accepted += 1;
      }
    }
  }
  // two-loop recursion on the coefficients of q = H G in {G, y_a, s_a}
  double gs[kMaxLbfgs], rho[kMaxLbfgs], alpha[kMaxLbfgs], qy[kMaxLbfgs], rs[kMaxLbfgs];
  for (int a = 0; a < c; ++a) {
    gs[a] = -S->tp[S->ord[a]] * gsE[a];
    rho[a] = 1.0 / S->SY[a][a];
    qy[a] = 0.0;
    rs[a] = 0.0;
  }
  for (int a = c - 1; a >= 0; --a) {
    double sq = gs[a];
    for (int b = 0; b < c; ++b) sq += qy[b] * S->SY[a][b];
    alpha[a] = rho[a] * sq;
    qy[a] -= alpha[a];
  }
  const double gam = c > 0 ? S->SY[c - 1][c - 1] / S->YY[c - 1][c - 1] : 1.0;
  const double rg = gam;
  for (int b = 0; b < c; ++b) qy[b] *= gam;
  for (int a = 0; a < c; ++a) {
    double yr = rg * gsY[a];
    for (int b = 0; b < c; ++b) yr += qy[b] * S->YY[a][b] + rs[b] * S->SY[b][a];
    const double beta = rho[a] * yr;
    rs[a] += alpha[a] - beta;
  }
  // descent test E . G > 0 from the same products
  double eg = rg * sc->tot[P_GG];
  for (int a = 0; a < c; ++a) eg += qy[a] * gsY[a] + rs[a] * gs[a];
  if (c > 0 && !(eg > 0.0)) {
    c = 0;
    S->resets += 1;
  }
  if (c == 0) {
    S->cg = 1.0;
  } else {
    S->cg = rg;
    for (int a = 0; a < c; ++a) {
      S->cy[a] = qy[a];
      S->ce[a] = -S->tp[S->ord[a]] * rs[a];
    }
  }
  S->cnt = c;
  S->cur = next;
  S->have = 1;
}

// ---- the direction and its line-search partials ----------------------------------

template <typename T, int LPR, int VEC, bool FULL>
__global__ void __launch_bounds__(kBlock)
k_lbfgs_combine(long n, int r, const T* __restrict__ R, const T* __restrict__ G, const double* __restrict__ y,
                const double* __restrict__ b, double sigma, const double* __restrict__ Av, LbfgsRing<RingT<T>> lb,
                double* __restrict__ part, const DevScalars* __restrict__ sc_base, BlockTab tab) {
  using V = typename Acc<T>::type;
  using RS = RingT<T>;
  const Rows ch = rows_of(n, tab);
  if (sc_base[ch.inst].flag) return;
  const LbfgsState* S = lb.s + ch.inst;
  const int c = S->cnt;
  const V cg = static_cast<V>(S->cg);
  const long xb = row_base(tab, ch.inst);
  R += xb;
  G += xb;
  RS* __restrict__ E = lb.e + (long)S->cur * lb.stride + xb;
  constexpr int RPB = kBlock / LPR;
  const int lane = threadIdx.x % LPR;
  const int slot = threadIdx.x / LPR;
  SplitAcc<NUM_P, LPR> acc;
  acc.zero();
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V ri[VEC], gi[VEC], e[VEC];
    load_frag<T, VEC, FULL>(R + i * r, lane, r, ri);
    load_frag<T, VEC, FULL>(G + i * r, lane, r, gi);
#pragma unroll
    for (int v = 0; v < VEC; ++v) e[v] = cg * gi[v];
    for (int a = 0; a < c; ++a) {
      const long off = (long)S->ord[a] * lb.stride + xb + i * r;
      const V ca = static_cast<V>(S->ce[a]), cb = static_cast<V>(S->cy[a]);
      V ev[VEC], yv[VEC];
      load_frag<RS, VEC, FULL>(lb.e + off, lane, r, ev);
      load_frag<RS, VEC, FULL>(lb.y + off, lane, r, yv);
#pragma unroll
      for (int v = 0; v < VEC; ++v) e[v] += ca * ev[v] + cb * yv[v];
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) e[v] = round_st<RS>(e[v]);  // the direction as stored
    store_frag<RS, VEC, FULL>(E + i * r, lane, r, e);
    // C R = G/2 + w R at the current point
    const double yi = y[i], ai = Av[i], ei = ai - b[i];
    const V wv = static_cast<V>(yi - sigma * ei);
    V ee = 0, ep = 0, re = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const V p = V(0.5) * gi[v] + wv * ri[v];
      ee += e[v] * e[v];
      ep += e[v] * p;
      re += ri[v] * e[v];
    }
    ee = group_sum<LPR>(ee);
    ep = group_sum<LPR>(ep);
    re = group_sum<LPR>(re);
    const double a1 = 2.0 * (double)re, a2 = (double)ee;
    acc.add(lane, P_GG, a2);
    acc.add(lane, P_GP, (double)ep);
    acc.add(lane, P_YA1, yi * a1);
    acc.add(lane, P_YA2, yi * a2);
    acc.add(lane, P_EA1, ei * a1);
    acc.add(lane, P_EA2, ei * a2);
    acc.add(lane, P_A1A1, a1 * a1);
    acc.add(lane, P_A1A2, a1 * a2);
    acc.add(lane, P_A2A2, a2 * a2);
    acc.add(lane, P_RG, (double)re);
  }
  acc.block_store(lane, part + part_slot(tab) * NUM_P);
}

__global__ void __launch_bounds__(kBlock)
k_fin_lsdir(const double* __restrict__ part, int nb, DevScalars* __restrict__ sc_base, LbfgsState* __restrict__ S_base,
            BlockTab tab) {
  DevScalars* sc = sc_base + blockIdx.x;
  LbfgsState* S = S_base + blockIdx.x;
  if (sc->flag) return;
  int b0, b1;
  inst_blocks(tab, blockIdx.x, nb, b0, b1);
  constexpr int K = 10;
  const int sl[K] = {P_GG, P_GP, P_YA1, P_YA2, P_EA1, P_EA2, P_A1A1, P_A1A2, P_A2A2, P_RG};
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int bi = b0 + threadIdx.x; bi < b1; bi += kBlock)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += part[(long)bi * NUM_P + sl[k]];
  __shared__ double tot[K];
  block_sum_store<K>(acc, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < K; ++k) sc->tot[sl[k]] = tot[k];
  S->ee = tot[0];
}

// ---- launchers ---------------------------------------------------------------------

void launch_lbfgs_reset(LbfgsState* s, int m, hipStream_t st, int count) {
  hipLaunchKernelGGL(k_lbfgs_reset, dim3(count), dim3(64), 0, st, s, m);
}

template <typename T>
void launch_lbfgs_dots(long len, int r, const T* G, const LbfgsRing<RingT<T>>& lb, double* part, int nb,
                       const DevScalars* sc, hipStream_t st, const BlockTab& tab) {
  hipLaunchKernelGGL((k_lbfgs_dots<T>), dim3(nb), dim3(kBlock), 0, st, len, r, G, lb, part, sc, tab);
}

void launch_fin_lbfgs(const double* part, int nb, const DevScalars* sc, LbfgsState* s, hipStream_t st,
                      const BlockTab& tab, int count) {
  hipLaunchKernelGGL(k_fin_lbfgs, dim3(count), dim3(kBlock), 0, st, part, nb, sc, s, tab);
}

template <typename T, int LPR, int VEC>
static void launch_combine_cfg(long n, int r, const T* R, const T* G, const double* y, const double* b, double sigma,
                               const double* Av, const LbfgsRing<RingT<T>>& lb, double* part,
                               const DevScalars* sc, int nblk, hipStream_t st, const BlockTab& tab) {
  if (r == LPR * VEC)
    hipLaunchKernelGGL((k_lbfgs_combine<T, LPR, VEC, true>), dim3(nblk), dim3(kBlock), 0, st, n, r, R, G, y, b,
                       sigma, Av, lb, part, sc, tab);
  else
    hipLaunchKernelGGL((k_lbfgs_combine<T, LPR, VEC, false>), dim3(nblk), dim3(kBlock), 0, st, n, r, R, G, y, b,
                       sigma, Av, lb, part, sc, tab);
}

template <typename T>
void launch_lbfgs_combine(long n, int r, int variant, const T* R, const T* G, const double* y, const double* b,
                          double sigma, const double* Av, const LbfgsRing<RingT<T>>& lb, double* part,
                          const DevScalars* sc, int nblk, hipStream_t st, const BlockTab& tab) {
  ALMBM_DISPATCH_DIAG(T, launch_combine_cfg, n, r, R, G, y, b, sigma, Av, lb, part, sc, nblk, st, tab);
}

void launch_fin_lsdir(const double* part, int nb, DevScalars* sc, LbfgsState* s, hipStream_t st,
                      const BlockTab& tab, int count) {
  hipLaunchKernelGGL(k_fin_lsdir, dim3(count), dim3(kBlock), 0, st, part, nb, sc, s, tab);
}

#define ALMBM_LBFGS_INST(T)                                                                               \
  template void launch_lbfgs_dots<T>(long, int, const T*, const LbfgsRing<RingT<T>>&, double*, int,       \
                                     const DevScalars*, hipStream_t, const BlockTab&);                     \
  template void launch_lbfgs_combine<T>(long, int, int, const T*, const T*, const double*, const double*,   \
                                        double, const double*, const LbfgsRing<RingT<T>>&, double*,          \
                                        const DevScalars*, int, hipStream_t, const BlockTab&);

ALMBM_LBFGS_INST(double)
ALMBM_LBFGS_INST(float)
ALMBM_LBFGS_INST(bf16)

}  // namespace almbm
