// Row kernels for the TRACE_EDGES constraint family: A_0 = c_tr I and, per
// edge e = {i, j}, A_{1+e} = (e_i e_j^T + e_j e_i^T)/2 (entry constraints as in
// the examples of Sec. 3.3 / Sec. 4.3; with C = -J they give the Lovasz-theta
// SDP).  Cost C = S + Diag(d) - j J.
//
// Pass 1 (SDDMM): a_{1+e} = <R_i, R_j> for every edge from the upper half of
//   the pattern (each edge once, edge order = position), w_e = y_e - sigma
//   (a_e - b_e), plus column sums 1^T R and ||R||^2 for the trace row and J.
// Pass 2 (SpMM): G_i = 2 (P_i - c_tr w_0 R_i - 1/2 sum_{j~i} w_{e(ij)} R_j) with
//   P_i = (S R)_i + d_i R_i - j (1^T R); the symmetric pattern carries edge ids.
// Pass 3 (line search): a1_e = <R_i,G_j> + <G_i,R_j>, a2_e = <G_i,G_j> over the
//   upper half and <G, (S + D) G>.
// The edge rows may carry their own penalty rho * sigma (the trace row keeps
// sigma): pass 1 forms w_e with it and weights the edge residual sums by rho,
// pass 3 weights the edge terms of the quartic by rho, so the finalizers'
// common factor sigma yields sigma on the trace row and rho sigma on the edges.
#include "spmm_row.hpp"
#include "quartic.hpp"

namespace almbm {

constexpr int kEdgePS = NUM_P + kMaxR;  // partial stride: scalars, then r column sums
constexpr int kEdgePre = 64;            // rows after the finalizers' first reduction stage

// out[c] = sum over blocks of the column-sum partials (c < r <= kMaxR), by the
// whole (single) block: P = kBlock / r threads per column take the blocks
// bi = j, j + P, ... and their P values are added in order of j, so the result
// does not depend on timing.  Every thread of the block must call it.
__device__ __forceinline__ void colsum_reduce(const double* __restrict__ part, int nb, int r, double* __restrict__ out) {
  __shared__ double buf[kBlock];
  const int P = kBlock / r;
  const int c = threadIdx.x % r, j = threadIdx.x / r;
  double a = 0.0;
  if (j < P)
    for (int bi = j; bi < nb; bi += P) a += part[(long)bi * kEdgePS + NUM_P + c];
  buf[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x < r) {
    double t = 0.0;
    for (int k = 0; k < P; ++k) t += buf[k * r + threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// out[q] = sum over blocks of the scalar partial part[b * kEdgePS + sl[q]], all K
// slots in one pass (each thread takes the blocks t, t + kBlock, ...; the block
// reduction is in fixed order).  Every thread of the (single) block must call it.
template <int K>
__device__ __forceinline__ void reduce_slots(const double* __restrict__ part, int nb, const int (&sl)[K],
                                             double (&out)[K]) {
  double acc[K];
#pragma unroll
  for (int q = 0; q < K; ++q) acc[q] = 0.0;
  for (int bi = threadIdx.x; bi < nb; bi += kBlock)
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] += part[(long)bi * kEdgePS + sl[q]];
  __shared__ double res[K];
  block_sum_store<K>(acc, res);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < K; ++q) out[q] = res[q];
  __syncthreads();
}

// Sum over the lanes of a block that share the same lane-in-row index (i.e.
// over row groups) of a VEC-wide fragment, deterministic; thread t < LPR of the
// first wave ends with the block totals for columns [t*VEC, t*VEC+VEC).
template <int LPR, int VEC>
__device__ __forceinline__ void block_colsum_store(double (&cs)[VEC], int r, double* __restrict__ out) {
  __shared__ double red[kBlock / kWave][LPR * VEC];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    double x = cs[v];
    for (int o = kWave / 2; o >= LPR; o >>= 1) x += __shfl_xor(x, o, kWave);
    cs[v] = x;
  }
  if (lane < LPR) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) red[wave][lane * VEC + v] = cs[v];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < LPR * VEC; c += kBlock) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += red[w][c];
    if (c < r) out[c] = t;
  }
}

template <typename T, int LPR, int VEC, bool FULL, int S>
__global__ void __launch_bounds__(kBlock)
k_edges_p1(EdgeAdj A, long n, int r, const T* __restrict__ R, const double* __restrict__ y,
           const double* __restrict__ b, double sigma, double* __restrict__ Av, double* __restrict__ wE,
           double* __restrict__ part, const DevScalars* __restrict__ sc, double rho) {
  using V = typename Acc<T>::type;
  if (sc && sc->flag) return;
  constexpr int RPB = kBlock / (LPR * S);
  const int lane = threadIdx.x % LPR;
  const int grp = (threadIdx.x / LPR) % S;
  const int slot = threadIdx.x / (LPR * S);
  SplitAcc<NUM_P, LPR> acc;
  acc.zero();
  double cs[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) cs[v] = 0.0;
  const RowChunk ch = row_chunk(n);
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V ri[VEC];
    load_frag<T, VEC, FULL>(R + i * r, lane, r, ri);
    V rr = 0;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      rr += ri[v] * ri[v];
      if (grp == 0) cs[v] += (double)ri[v];
    }
    rr = group_sum<LPR>(rr);
    const int k0 = A.urp[i], k1 = A.urp[i + 1];
    // kUnroll neighbour rows in flight per group (entries past the row end
    // gather row i itself and are skipped), edges taken in order
    for (int k = k0 + grp; k < k1; k += S * kUnroll) {
      int jj[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int kk = k + u * S;
        jj[u] = kk < k1 ? A.uci[kk] : (int)i;
      }
      V rj[kUnroll][VEC];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) load_frag<T, VEC, FULL>(R + (long)jj[u] * r, lane, r, rj[u]);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int kk = k + u * S;
        if (kk >= k1) break;
        V s = 0;
#pragma unroll
        for (int v = 0; v < VEC; ++v) s += ri[v] * rj[u][v];
        s = group_sum<LPR>(s);
        const double a = s, be = b[1 + kk], ye = y[1 + kk];
        const double e = a - be;
        if (lane == 0) {
          if (Av) Av[1 + kk] = a;
          wE[kk] = ye - rho * sigma * e;
        }
        acc.add(lane, P_YBMA, ye * (be - a));
        acc.add(lane, P_EE, rho * e * e);
      }
    }
    if (grp == 0) acc.add(lane, P_RR, (double)rr);
  }
  acc.block_store(lane, part + (long)blockIdx.x * kEdgePS);
  block_colsum_store<LPR, VEC>(cs, r, part + (long)blockIdx.x * kEdgePS + NUM_P);
}

// Finalize of pass 1: trace row, w_0, column sums; writes Av[0].
__global__ void __launch_bounds__(kBlock)
k_fin_edges1(const double* __restrict__ part, int nb, int r, DevScalars* __restrict__ sc, const double* __restrict__ y,
             const double* __restrict__ b, double sigma, double c_tr, double* __restrict__ Av) {
  if (sc->flag) return;
  // scalars
  double tot3[3];
  const int sl[3] = {P_YBMA, P_EE, P_RR};
  reduce_slots<3>(part, nb, sl, tot3);
  colsum_reduce(part, nb, r, sc->colsum);
  if (threadIdx.x == 0) {
    const double rr = tot3[2];
    const double a0 = c_tr * rr;
    const double e0 = a0 - b[0];
    sc->a0 = a0;
    sc->w0 = y[0] - sigma * e0;
    if (Av) Av[0] = a0;
    sc->tot[P_YBMA] = tot3[0] + y[0] * (b[0] - a0);
    sc->tot[P_EE] = tot3[1] + e0 * e0;
    sc->tot[P_RR] = rr;
  }
}

// Pass 2: P = C R, gradient and its partials.  If G_in is given, the direction
// is read instead of computed (line-search API) and nothing is written.
template <typename T, int LPR, int VEC, bool FULL, int S>
__global__ void __launch_bounds__(kBlock)
k_edges_p2(Cost<typename Acc<T>::type> C, EdgeAdj A, int r, const T* __restrict__ R,
           const double* __restrict__ wE, double c_tr, double j_coef, const T* __restrict__ G_in,
           T* __restrict__ G, double* __restrict__ part, const DevScalars* __restrict__ sc) {
  using V = typename Acc<T>::type;
  if (sc->flag) return;
  constexpr int RPB = kBlock / (LPR * S);
  const int lane = threadIdx.x % LPR;
  const int grp = (threadIdx.x / LPR) % S;
  const int slot = threadIdx.x / (LPR * S);
  SplitAcc<NUM_P, LPR> acc;
  acc.zero();
  double gcs[VEC];
  V jcs[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    gcs[v] = 0.0;
    const int c = lane * VEC + v;
    jcs[v] = (c < r && j_coef != 0.0) ? static_cast<V>(j_coef * sc->colsum[c]) : V(0);
  }
  const V cw0 = static_cast<V>(c_tr * sc->w0);
  const RowChunk ch = row_chunk(C.n);
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V ri[VEC], p[VEC], ad[VEC];
    load_frag<T, VEC, FULL>(R + i * r, lane, r, ri);
    if (grp == 0) {
      spmm_row<T, LPR, VEC, FULL>(C, i, lane, r, R, ri, p);
    } else {
#pragma unroll
      for (int v = 0; v < VEC; ++v) p[v] = V(0);
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      p[v] -= jcs[v];
      ad[v] = grp == 0 ? cw0 * ri[v] : V(0);
    }
    const int k0 = A.rp[i], k1 = A.rp[i + 1];
    for (int k = k0 + grp; k < k1; k += S) {
      const int j = A.ci[k];
      const V we = static_cast<V>(0.5 * wE[A.eid[k]]);
      V rj[VEC];
      load_frag<T, VEC, FULL>(R + (long)j * r, lane, r, rj);
#pragma unroll
      for (int v = 0; v < VEC; ++v) ad[v] += we * rj[v];
    }
    // the S groups of the row add their shares in a fixed butterfly order
#pragma unroll
    for (int o = LPR; o < LPR * S; o <<= 1)
#pragma unroll
      for (int v = 0; v < VEC; ++v) ad[v] += __shfl_xor(ad[v], o, kWave);
    if (grp == 0) {  // the row's own terms, once
      V g[VEC];
      if (G_in) {
        load_frag<T, VEC, FULL>(G_in + i * r, lane, r, g);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) g[v] = round_st<T>(V(2) * (p[v] - ad[v]));
        if (G) store_frag<T, VEC, FULL>(G + i * r, lane, r, g);
      }
      V rp = 0, gg = 0, gp = 0, rg = 0;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        rp += ri[v] * p[v];
        gg += g[v] * g[v];
        gp += g[v] * p[v];
        rg += ri[v] * g[v];
        gcs[v] += (double)g[v];
      }
      rp = group_sum<LPR>(rp);
      gg = group_sum<LPR>(gg);
      gp = group_sum<LPR>(gp);
      rg = group_sum<LPR>(rg);
      acc.add(lane, P_C0, (double)rp);
      acc.add(lane, P_GG, (double)gg);
      acc.add(lane, P_GP, (double)gp);
      acc.add(lane, P_RG, (double)rg);
    }
  }
  acc.block_store(lane, part + (long)blockIdx.x * kEdgePS);
  block_colsum_store<LPR, VEC>(gcs, r, part + (long)blockIdx.x * kEdgePS + NUM_P);
}

// Finalize of pass 2: objective and (mode 1) the inner stop test.
__global__ void __launch_bounds__(kBlock)
k_fin_edges2(const double* __restrict__ part, int nb, int r, DevScalars* __restrict__ sc, double sigma, int mode,
             double* __restrict__ f_out) {
  if (sc->flag) return;
  double tot4[4];
  const int sl[4] = {P_C0, P_GG, P_GP, P_RG};
  reduce_slots<4>(part, nb, sl, tot4);
  colsum_reduce(part, nb, r, sc->gcolsum);
  if (threadIdx.x != 0) return;
  sc->tot[P_C0] = tot4[0];
  sc->tot[P_GG] = tot4[1];
  sc->tot[P_GP] = tot4[2];
  sc->tot[P_RG] = tot4[3];
  const double f = tot4[0] + sc->tot[P_YBMA] + 0.5 * sigma * sc->tot[P_EE];
  sc->f = f;
  if (!isfinite(f) || !isfinite(tot4[1])) sc->numeric_error = 1;
  if (f_out) *f_out = f;
  if (mode == 1) {
    const double lhs = sqrt(tot4[1]) * sqrt(sc->tot[P_RR]);
    if (sc->iter >= sc->max_inner) sc->flag = 2;
    else if (lhs <= sc->tol * (1.0 + fabs(tot4[0])) || !isfinite(lhs)) sc->flag = 1;
    else sc->iter += 1;
  }
}

// Pass 3: line-search partials over the edges and <G, (S + D) G>.
template <typename T, int LPR, int VEC, bool FULL, int S>
__global__ void __launch_bounds__(kBlock)
k_edges_p3(Cost<typename Acc<T>::type> C, EdgeAdj A, int r, const T* __restrict__ R, const T* __restrict__ G,
           const double* __restrict__ y, const double* __restrict__ b, const double* __restrict__ Av,
           double* __restrict__ part, const DevScalars* __restrict__ sc, double rho) {
  using V = typename Acc<T>::type;
  if (sc->flag) return;
  constexpr int RPB = kBlock / (LPR * S);
  const int lane = threadIdx.x % LPR;
  const int grp = (threadIdx.x / LPR) % S;
  const int slot = threadIdx.x / (LPR * S);
  SplitAcc<NUM_P, LPR> acc;
  acc.zero();
  const RowChunk ch = row_chunk(C.n);
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + slot;
    if (i >= ch.hi) break;
    V ri[VEC], gi[VEC], q[VEC];
    load_frag<T, VEC, FULL>(R + i * r, lane, r, ri);
    load_frag<T, VEC, FULL>(G + i * r, lane, r, gi);
    if (grp == 0) {
      spmm_row<T, LPR, VEC, FULL>(C, i, lane, r, G, gi, q);
      V gq = 0;
#pragma unroll
      for (int v = 0; v < VEC; ++v) gq += gi[v] * q[v];
      gq = group_sum<LPR>(gq);
      acc.add(lane, P_C2, (double)gq);
    }
    const int k0 = A.urp[i], k1 = A.urp[i + 1];
    constexpr int U3 = kUnroll / 2;  // two rows (R_j, G_j) per edge
    for (int k = k0 + grp; k < k1; k += S * U3) {
      int jj[U3];
#pragma unroll
      for (int u = 0; u < U3; ++u) {
        const int kk = k + u * S;
        jj[u] = kk < k1 ? A.uci[kk] : (int)i;
      }
      V rj[U3][VEC], gj[U3][VEC];
#pragma unroll
      for (int u = 0; u < U3; ++u) {
        load_frag<T, VEC, FULL>(R + (long)jj[u] * r, lane, r, rj[u]);
        load_frag<T, VEC, FULL>(G + (long)jj[u] * r, lane, r, gj[u]);
      }
#pragma unroll
      for (int u = 0; u < U3; ++u) {
      const int kk = k + u * S;
      if (kk >= k1) break;
      V a1 = 0, a2 = 0;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        a1 += ri[v] * gj[u][v] + gi[v] * rj[u][v];
        a2 += gi[v] * gj[u][v];
      }
      a1 = group_sum<LPR>(a1);
      a2 = group_sum<LPR>(a2);
      const double ye = y[1 + kk], e = Av[1 + kk] - b[1 + kk];
      const double d1 = a1, d2 = a2;
      acc.add(lane, P_YA1, ye * d1);
      acc.add(lane, P_YA2, ye * d2);
      acc.add(lane, P_EA1, rho * e * d1);
      acc.add(lane, P_EA2, rho * e * d2);
      acc.add(lane, P_A1A1, rho * d1 * d1);
      acc.add(lane, P_A1A2, rho * d1 * d2);
      acc.add(lane, P_A2A2, rho * d2 * d2);
      }
    }
  }
  acc.block_store(lane, part + (long)blockIdx.x * kEdgePS);
}

// Finalize of pass 3: add the trace row and the -jJ terms, then the step.

__global__ void __launch_bounds__(kBlock)
k_fin_edges3(const double* __restrict__ part, int nb, int r, DevScalars* __restrict__ sc, const double* __restrict__ y,
             const double* __restrict__ b, double sigma, double c_tr, double j_coef, int mode,
             double* __restrict__ coeffs_out, double* __restrict__ t_out) {
  if (mode == 1 && sc->flag) return;
  const int sl[8] = {P_C2, P_YA1, P_YA2, P_EA1, P_EA2, P_A1A1, P_A1A2, P_A2A2};
  double tot8[8];
  reduce_slots<8>(part, nb, sl, tot8);
  if (threadIdx.x != 0) return;
  double gj2 = 0.0;
  for (int c = 0; c < r; ++c) gj2 += sc->gcolsum[c] * sc->gcolsum[c];
  const double a1_0 = 2.0 * c_tr * sc->tot[P_RG];
  const double a2_0 = c_tr * sc->tot[P_GG];
  const double e0 = sc->a0 - b[0];
  double* tot = sc->tot;
  tot[P_C2] = tot8[0] - j_coef * gj2;
  tot[P_YA1] = tot8[1] + y[0] * a1_0;
  tot[P_YA2] = tot8[2] + y[0] * a2_0;
  tot[P_EA1] = tot8[3] + e0 * a1_0;
  tot[P_EA2] = tot8[4] + e0 * a2_0;
  tot[P_A1A1] = tot8[5] + a1_0 * a1_0;
  tot[P_A1A2] = tot8[6] + a1_0 * a2_0;
  tot[P_A2A2] = tot8[7] + a2_0 * a2_0;
  double k[5];
  quartic_coeffs(tot, sigma, k);
  for (int s = 0; s < 5; ++s) sc->coeffs[s] = k[s];
  double t = (mode == 1 && sc->step_rule == 1) ? sc->eta_fixed : quartic_argmin(k);
  if (!isfinite(t)) {
    t = 0.0;
    sc->numeric_error = 1;
  }
  sc->t = t;
  if (coeffs_out)
    for (int s = 0; s < 5; ++s) coeffs_out[s] = k[s];
  if (t_out) *t_out = t;
}

// ---- launchers -----------------------------------------------------------------

#define ALMBM_DISPATCH_EDGES(T, FN, ...)                                \
  do {                                                                  \
    if constexpr (sizeof(T) == 8) {                                     \
      if (r <= 4) FN<T, 4, 1>(__VA_ARGS__);                             \
      else if (r <= 8) FN<T, 8, 1>(__VA_ARGS__);                        \
      else if (r <= 16) FN<T, 8, 2>(__VA_ARGS__);                       \
      else if (r <= 32) FN<T, 8, 4>(__VA_ARGS__);                       \
      else if (r <= 64) FN<T, 16, 4>(__VA_ARGS__);                      \
      else FN<T, 32, 4>(__VA_ARGS__);                                   \
    } else if constexpr (sizeof(T) == 4) {                              \
      if (r <= 4) FN<T, 4, 1>(__VA_ARGS__);                             \
      else if (r <= 8) FN<T, 4, 2>(__VA_ARGS__);                        \
      else if (r <= 16) FN<T, 4, 4>(__VA_ARGS__);                       \
      else if (r <= 32) { if (variant == 1) FN<T, 4, 8>(__VA_ARGS__); else FN<T, 8, 4>(__VA_ARGS__); } \
      else if (r <= 64) FN<T, 16, 4>(__VA_ARGS__);                      \
      else FN<T, 32, 4>(__VA_ARGS__);                                   \
    } else {                                                            \
      if (r <= 4) FN<T, 2, 2>(__VA_ARGS__);                             \
      else if (r <= 8) FN<T, 2, 4>(__VA_ARGS__);                        \
      else if (r <= 16) FN<T, 2, 8>(__VA_ARGS__);                       \
      else if (r <= 32) FN<T, 4, 8>(__VA_ARGS__);                       \
      else if (r <= 64) FN<T, 8, 8>(__VA_ARGS__);                       \
      else FN<T, 16, 8>(__VA_ARGS__);                                   \
    }                                                                   \
  } while (0)

template <typename T, int LPR, int VEC>
static void p1_cfg(const EdgeAdj& A, long n, int r, const T* R, const double* y, const double* b, double sigma,
                   double* Av, double* wE, double* part, const DevScalars* sc, int nblk, hipStream_t st, double rho) {
  const bool split = A.avg_deg >= 8.f * (kWave / LPR);
  if (r == LPR * VEC)
    {
      if (split)
        hipLaunchKernelGGL((k_edges_p1<T, LPR, VEC, true, kWave / LPR>), dim3(nblk), dim3(kBlock), 0, st, A, n, r, R, y, b, sigma, Av, wE, part, sc, rho);
      else
        hipLaunchKernelGGL((k_edges_p1<T, LPR, VEC, true, 1>), dim3(nblk), dim3(kBlock), 0, st, A, n, r, R, y, b, sigma, Av, wE, part, sc, rho);
    }
  else
    {
      if (split)
        hipLaunchKernelGGL((k_edges_p1<T, LPR, VEC, false, kWave / LPR>), dim3(nblk), dim3(kBlock), 0, st, A, n, r, R, y, b, sigma, Av, wE, part, sc, rho);
      else
        hipLaunchKernelGGL((k_edges_p1<T, LPR, VEC, false, 1>), dim3(nblk), dim3(kBlock), 0, st, A, n, r, R, y, b, sigma, Av, wE, part, sc, rho);
    }
}
template <typename T, int LPR, int VEC>
static void p2_cfg(const Cost<typename Acc<T>::type>& C, const EdgeAdj& A, int r, const T* R, const double* wE,
                   double c_tr, double j_coef, const T* G_in, T* G, double* part, const DevScalars* sc, int nblk,
                   hipStream_t st) {
  const bool split = A.avg_deg >= 8.f * (kWave / LPR);
  if (r == LPR * VEC)
    {
      if (split)
        hipLaunchKernelGGL((k_edges_p2<T, LPR, VEC, true, kWave / LPR>), dim3(nblk), dim3(kBlock), 0, st, C, A, r, R, wE, c_tr, j_coef, G_in, G, part, sc);
      else
        hipLaunchKernelGGL((k_edges_p2<T, LPR, VEC, true, 1>), dim3(nblk), dim3(kBlock), 0, st, C, A, r, R, wE, c_tr, j_coef, G_in, G, part, sc);
    }
  else
    {
      if (split)
        hipLaunchKernelGGL((k_edges_p2<T, LPR, VEC, false, kWave / LPR>), dim3(nblk), dim3(kBlock), 0, st, C, A, r, R, wE, c_tr, j_coef, G_in, G, part, sc);
      else
        hipLaunchKernelGGL((k_edges_p2<T, LPR, VEC, false, 1>), dim3(nblk), dim3(kBlock), 0, st, C, A, r, R, wE, c_tr, j_coef, G_in, G, part, sc);
    }
}
template <typename T, int LPR, int VEC>
static void p3_cfg(const Cost<typename Acc<T>::type>& C, const EdgeAdj& A, int r, const T* R, const T* G,
                   const double* y, const double* b, const double* Av, double* part, const DevScalars* sc, int nblk,
                   hipStream_t st, double rho) {
  const bool split = A.avg_deg >= 8.f * (kWave / LPR);
  if (r == LPR * VEC)
    {
      if (split)
        hipLaunchKernelGGL((k_edges_p3<T, LPR, VEC, true, kWave / LPR>), dim3(nblk), dim3(kBlock), 0, st, C, A, r, R, G, y, b, Av, part, sc, rho);
      else
        hipLaunchKernelGGL((k_edges_p3<T, LPR, VEC, true, 1>), dim3(nblk), dim3(kBlock), 0, st, C, A, r, R, G, y, b, Av, part, sc, rho);
    }
  else
    {
      if (split)
        hipLaunchKernelGGL((k_edges_p3<T, LPR, VEC, false, kWave / LPR>), dim3(nblk), dim3(kBlock), 0, st, C, A, r, R, G, y, b, Av, part, sc, rho);
      else
        hipLaunchKernelGGL((k_edges_p3<T, LPR, VEC, false, 1>), dim3(nblk), dim3(kBlock), 0, st, C, A, r, R, G, y, b, Av, part, sc, rho);
    }
}

template <typename T>
void launch_edges_p1(const EdgeAdj& A, long n, int r, int variant, const T* R, const double* y, const double* b,
                     double sigma, double* Av, double* wE, double* part, const DevScalars* sc, int nblk,
                     hipStream_t st, double rho) {
  ALMBM_DISPATCH_EDGES(T, p1_cfg, A, n, r, R, y, b, sigma, Av, wE, part, sc, nblk, st, rho);
}
template <typename T>
void launch_edges_p2(const Cost<typename Acc<T>::type>& C, const EdgeAdj& A, int r, int variant, const T* R,
                     const double* wE, double c_tr, double j_coef, const T* G_in, T* G, double* part,
                     const DevScalars* sc, int nblk, hipStream_t st) {
  ALMBM_DISPATCH_EDGES(T, p2_cfg, C, A, r, R, wE, c_tr, j_coef, G_in, G, part, sc, nblk, st);
}
template <typename T>
void launch_edges_p3(const Cost<typename Acc<T>::type>& C, const EdgeAdj& A, int r, int variant, const T* R,
                     const T* G, const double* y, const double* b, const double* Av, double* part,
                     const DevScalars* sc, int nblk, hipStream_t st, double rho) {
  ALMBM_DISPATCH_EDGES(T, p3_cfg, C, A, r, R, G, y, b, Av, part, sc, nblk, st, rho);
}

// First stage of the finalizers' reductions: block k of kEdgePre sums the
// partial rows [k nb / kEdgePre, (k+1) nb / kEdgePre) of the first ncols
// columns in order into row k of out, so the one-block finalizer then reduces
// kEdgePre rows instead of nb (thousands at the Lovasz and completion shapes).
__global__ void __launch_bounds__(kBlock)
k_edges_prereduce(const double* __restrict__ part, int nb, int ncols, double* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= ncols) return;
  const long lo = (long)blockIdx.x * nb / gridDim.x, hi = (long)(blockIdx.x + 1) * nb / gridDim.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  long bi = lo;
  for (; bi + 4 <= hi; bi += 4) {
    a0 += part[bi * kEdgePS + c];
    a1 += part[(bi + 1) * kEdgePS + c];
    a2 += part[(bi + 2) * kEdgePS + c];
    a3 += part[(bi + 3) * kEdgePS + c];
  }
  for (; bi < hi; ++bi) a0 += part[bi * kEdgePS + c];
  out[(long)blockIdx.x * kEdgePS + c] = (a0 + a1) + (a2 + a3);
}

static const double* prereduce(const double* part, int& nb, int r, double* part2, hipStream_t st) {
  if (!part2 || nb <= kEdgePre) return part;
  hipLaunchKernelGGL(k_edges_prereduce, dim3(kEdgePre), dim3(kBlock), 0, st, part, nb, NUM_P + r, part2);
  nb = kEdgePre;
  return part2;
}

void launch_fin_edges1(const double* part, int nb, int r, DevScalars* sc, const double* y, const double* b,
                       double sigma, double c_tr, double* Av, hipStream_t st, double* part2) {
  part = prereduce(part, nb, r, part2, st);
  hipLaunchKernelGGL(k_fin_edges1, dim3(1), dim3(kBlock), 0, st, part, nb, r, sc, y, b, sigma, c_tr, Av);
}
void launch_fin_edges2(const double* part, int nb, int r, DevScalars* sc, double sigma, int mode, double* f_out,
                       hipStream_t st, double* part2) {
  part = prereduce(part, nb, r, part2, st);
  hipLaunchKernelGGL(k_fin_edges2, dim3(1), dim3(kBlock), 0, st, part, nb, r, sc, sigma, mode, f_out);
}
void launch_fin_edges3(const double* part, int nb, int r, DevScalars* sc, const double* y, const double* b,
                       double sigma, double c_tr, double j_coef, int mode, double* coeffs_out, double* t_out,
                       hipStream_t st, double* part2) {
  part = prereduce(part, nb, r, part2, st);
  hipLaunchKernelGGL(k_fin_edges3, dim3(1), dim3(kBlock), 0, st, part, nb, r, sc, y, b, sigma, c_tr, j_coef, mode,
                     coeffs_out, t_out);
}

#define ALMBM_INST_E(T)                                                                                        \
  template void launch_edges_p1<T>(const EdgeAdj&, long, int, int, const T*, const double*, const double*, double, \
                                   double*, double*, double*, const DevScalars*, int, hipStream_t, double);    \
  template void launch_edges_p2<T>(const Cost<Acc<T>::type>&, const EdgeAdj&, int, int, const T*, const double*, \
                                   double, double, const T*, T*, double*, const DevScalars*, int, hipStream_t); \
  template void launch_edges_p3<T>(const Cost<Acc<T>::type>&, const EdgeAdj&, int, int, const T*, const T*,     \
                                   const double*, const double*, const double*, double*, const DevScalars*, int, \
                                   hipStream_t, double);

ALMBM_INST_E(double)
ALMBM_INST_E(float)
ALMBM_INST_E(bf16)

}  // namespace almbm
