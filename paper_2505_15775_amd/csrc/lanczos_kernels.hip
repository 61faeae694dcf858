// Lanczos for lambda_min of the dual slack Z(y) = C - A*(y) (Sec. 1.2), used
// by the KKT measure of Sec. 6 and the rank test of Alg. 1.  Everything in FP64:
// the matrix-free product, dot products and the full reorthogonalisation
// (classical Gram-Schmidt applied twice) against the stored basis Q
// (column-major, n x (k+1), leading dimension ldq).
#include "launch.hpp"

namespace almbm {

constexpr int kSpmvLpr = 4;  // lanes per row in the slack product (avg degree ~ 8)

// out_i = (Z(y) x)_i.  DIAG: (d_i - y_i) x_i + sum_k S_ik x_k.
// TRACE_EDGES: (S x)_i + d_i x_i - j (1^T x) - c_tr y_0 x_i - 1/2 sum_{k~i} y_{1+e(ik)} x_k.
__global__ void __launch_bounds__(kBlock)
k_slack_mv(Cost<double> C, int cons_kind, EdgeAdj A, const double* __restrict__ y, double c_tr, double j_coef,
           const DevScalars* __restrict__ sc, const double* __restrict__ x, double* __restrict__ out) {
  constexpr int L = kSpmvLpr;
  const long i = ((long)blockIdx.x * kBlock + threadIdx.x) / L;
  const int lane = threadIdx.x % L;
  if (i >= C.n) return;
  double acc = 0.0;
  long k0 = 0, k1 = 0;
  if (C.ell > 0) {
    k0 = i * (long)C.ell;
    k1 = k0 + C.ell;
  } else if (C.rp) {
    k0 = C.rp[i];
    k1 = C.rp[i + 1];
  }
  if (C.nh > 0 && k1 - k0 > C.hthr) {  // hub row: sum precomputed by k_hub_rows
    if (lane == 0) acc = C.hsum[hub_index(C, i)];
  } else {
    for (long k = k0 + lane; k < k1; k += L) acc += C.cv[k] * x[C.ci[k]];
  }
  if (cons_kind == 1) {
    const int a0 = A.rp[i], a1 = A.rp[i + 1];
    for (int k = a0 + lane; k < a1; k += L) acc -= 0.5 * y[1 + A.eid[k]] * x[A.ci[k]];
  }
  acc = group_sum<L>(acc);
  if (lane == 0) {
    const double xi = x[i];
    double d = C.dg ? C.dg[i] : 0.0;
    if (cons_kind == 0) d -= y[i];
    else d -= c_tr * y[0];
    double v = acc + d * xi;
    if (j_coef != 0.0) v -= j_coef * sc->qsum;
    out[i] = v;
  }
}

// The same product over the rows of a block table (batched mode: only the
// blocks of the instances still running).
__global__ void __launch_bounds__(kBlock)
k_slack_mv_tab(Cost<double> C, const double* __restrict__ y, const double* __restrict__ x, double* __restrict__ out,
               BlockTab tab) {
  constexpr int L = kSpmvLpr;
  constexpr int RPB = kBlock / L;
  const Rows ch = rows_of(C.n, tab);
  const int lane = threadIdx.x % L;
  for (long base = ch.lo; base < ch.hi; base += RPB) {
    const long i = base + threadIdx.x / L;
    double acc = 0.0;
    if (i < ch.hi) {
      const long k0 = C.rp ? C.rp[i] : 0, k1 = C.rp ? C.rp[i + 1] : 0;
      for (long k = k0 + lane; k < k1; k += L) acc += C.cv[k] * x[C.ci[k]];
    }
    acc = group_sum<L>(acc);
    if (i < ch.hi && lane == 0) out[i] = acc + ((C.dg ? C.dg[i] : 0.0) - y[i]) * x[i];
  }
}

// partials[b][c] = sum over the block's rows of Q[c][i] * w[i], c < ncol.
// Wave w of the block handles columns c = w, w+4, ...; lanes stride the rows.
__global__ void __launch_bounds__(kBlock)
k_dots(long n, int ncol, const double* __restrict__ Q, long ldq, const double* __restrict__ w,
       double* __restrict__ part, int pstride, BlockTab tab) {
  const Rows ch = rows_of(n, tab);
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  for (int c = wave; c < ncol; c += kBlock / kWave) {
    const double* q = Q + (long)c * ldq;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    long i = ch.lo + lane;
    for (; i + 3 * kWave < ch.hi; i += 4 * kWave) {
      a0 += q[i] * w[i];
      a1 += q[i + kWave] * w[i + kWave];
      a2 += q[i + 2 * kWave] * w[i + 2 * kWave];
      a3 += q[i + 3 * kWave] * w[i + 3 * kWave];
    }
    for (; i < ch.hi; i += kWave) a0 += q[i] * w[i];
    double a = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) part[part_slot(tab) * pstride + c] = a;
  }
}

// h[q][c] = sum of the block partials of column c over instance q's blocks
// (grid: columns x instances, fixed order).
__global__ void __launch_bounds__(kBlock)
k_fin_dots(const double* __restrict__ part, int nb, int pstride, int ncol, double* __restrict__ h, int hstride,
           BlockTab tab) {
  const int c = blockIdx.x, q = blockIdx.y;
  if (c >= ncol) return;
  int b0, b1;
  inst_blocks(tab, q, nb, b0, b1);
  double acc[1] = {0.0};
  for (int b = b0 + threadIdx.x; b < b1; b += kBlock) acc[0] += part[(long)b * pstride + c];
  block_sum_store<1>(acc, h + (long)q * hstride + c);
}

// w_i -= sum_c Q[c][i] h[c]; partial ||w||^2 per block.
__global__ void __launch_bounds__(kBlock)
k_sub(long n, int ncol, const double* __restrict__ Q, long ldq, const double* __restrict__ h, int hstride,
      double* __restrict__ w, double* __restrict__ part, BlockTab tab) {
  const Rows ch = rows_of(n, tab);
  __shared__ double hs[512 + 1];
  for (int c = threadIdx.x; c < ncol; c += kBlock) hs[c] = h[(long)ch.inst * hstride + c];
  __syncthreads();
  double acc[1] = {0.0};
  for (long i = ch.lo + threadIdx.x; i < ch.hi; i += kBlock) {
    double v = w[i];
    for (int c = 0; c < ncol; ++c) v -= Q[(long)c * ldq + i] * hs[c];
    w[i] = v;
    acc[0] += v * v;
  }
  block_sum_store<1>(acc, part + part_slot(tab));
}

// Tridiagonal entries after the two projections: alpha_j = h1[j] + h2[j],
// beta_j = ||w||.
__global__ void __launch_bounds__(kBlock)
k_fin_ab(const double* __restrict__ part, int nb, const double* __restrict__ h1, const double* __restrict__ h2,
         int hstride, int j, double* __restrict__ alpha, double* __restrict__ beta, int astride, BlockTab tab) {
  const int q = blockIdx.x;
  int b0, b1;
  inst_blocks(tab, q, nb, b0, b1);
  h1 += (long)q * hstride;
  h2 += (long)q * hstride;
  alpha += (long)q * astride;
  beta += (long)q * astride;
  __shared__ double red[kBlock / kWave];
  double a = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += kBlock) a += part[b];
  a = wave_sum(a);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
    alpha[j] = h1[j] + h2[j];
    beta[j] = sqrt(t);
  }
}

// q = w / beta (beta > 0), partial sums of q for the -jJ term.
__global__ void __launch_bounds__(kBlock)
k_scale(long n, const double* __restrict__ w, const double* __restrict__ beta_ptr, int bstride, double* __restrict__ q,
        double* __restrict__ part, BlockTab tab) {
  const Rows ch = rows_of(n, tab);
  const double beta = beta_ptr[(long)ch.inst * bstride];
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  double acc[1] = {0.0};
  for (long i = ch.lo + threadIdx.x; i < ch.hi; i += kBlock) {
    const double v = w[i] * inv;
    q[i] = v;
    acc[0] += v;
  }
  block_sum_store<1>(acc, part + part_slot(tab));
}

__global__ void __launch_bounds__(kBlock)
k_fin_sum(const double* __restrict__ part, int nb, double* __restrict__ out, int ostride, int do_sqrt, BlockTab tab) {
  const int q = blockIdx.x;
  int b0, b1;
  inst_blocks(tab, q, nb, b0, b1);
  out += (long)q * ostride;
  __shared__ double red[kBlock / kWave];
  double a = 0.0;
  for (int b = b0 + threadIdx.x; b < b1; b += kBlock) a += part[b];
  a = wave_sum(a);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
    *out = do_sqrt ? sqrt(t) : t;
  }
}

// Start vector: counter-based uniform entries, partial ||x||^2.
__global__ void __launch_bounds__(kBlock)
k_rand(long n, uint64_t seed, double* __restrict__ x, double* __restrict__ part, BlockTab tab) {
  const Rows ch = rows_of(n, tab);
  double acc[1] = {0.0};
  for (long i = ch.lo + threadIdx.x; i < ch.hi; i += kBlock) {
    const double v = counter_uniform(seed, (uint64_t)i);
    x[i] = v;
    acc[0] += v * v;
  }
  block_sum_store<1>(acc, part + part_slot(tab));
}

// Warm start of a Lanczos pass: x = v + eps x / ||x|| per instance (x holds a
// random vector whose per-instance norm is at norms[inst * nstride], v the
// previous unit Ritz vector); partial ||x||^2.  The random share keeps every
// eigenvector in the start, so a bottom eigenvector that moved away from v is
// still found.
__global__ void __launch_bounds__(kBlock)
k_mix(long n, double eps, const double* __restrict__ v, double* __restrict__ x, const double* __restrict__ norms,
      int nstride, double* __restrict__ part, BlockTab tab) {
  const Rows ch = rows_of(n, tab);
  const double a = eps / fmax(norms[(long)ch.inst * nstride], 1e-300);
  double acc[1] = {0.0};
  for (long i = ch.lo + threadIdx.x; i < ch.hi; i += kBlock) {
    const double t = v[i] + a * x[i];
    x[i] = t;
    acc[0] += t * t;
  }
  block_sum_store<1>(acc, part + part_slot(tab));
}

// v = sum_c Q[c] s[c]; partial ||v||^2.
__global__ void __launch_bounds__(kBlock)
k_combine(long n, int ncol, const double* __restrict__ Q, long ldq, const double* __restrict__ s, int sstride,
          double* __restrict__ v, double* __restrict__ part, BlockTab tab, const int32_t* __restrict__ ncols) {
  const Rows ch = rows_of(n, tab);
  // per-instance basis sizes: columns past an instance's own count were not
  // written for its rows in this pass
  if (ncols && ncols[ch.inst] < ncol) ncol = ncols[ch.inst];
  __shared__ double ss[512 + 1];
  for (int c = threadIdx.x; c < ncol; c += kBlock) ss[c] = s[(long)ch.inst * sstride + c];
  __syncthreads();
  double acc[1] = {0.0};
  for (long i = ch.lo + threadIdx.x; i < ch.hi; i += kBlock) {
    double a = 0.0;
    for (int c = 0; c < ncol; ++c) a += Q[(long)c * ldq + i] * ss[c];
    v[i] = a;
    acc[0] += a * a;
  }
  block_sum_store<1>(acc, part + part_slot(tab));
}

// partial ||z - theta v||^2 (residual of the Ritz pair).
__global__ void __launch_bounds__(kBlock)
k_resid(long n, const double* __restrict__ z, const double* __restrict__ v, double theta,
        const double* __restrict__ thetas, double* __restrict__ part, BlockTab tab) {
  const Rows ch = rows_of(n, tab);
  if (thetas) theta = thetas[ch.inst];
  double acc[1] = {0.0};
  for (long i = ch.lo + threadIdx.x; i < ch.hi; i += kBlock) {
    const double d = z[i] - theta * v[i];
    acc[0] += d * d;
  }
  block_sum_store<1>(acc, part + part_slot(tab));
}

// sum_i x_i^4 (DIAG) or sum over edges of (x_i x_j)^2 (TRACE_EDGES): the
// curvature ||A(v v^T)||^2 of the rank-one step, without the trace row.
__global__ void __launch_bounds__(kBlock)
k_quartic_norm(long n, int cons_kind, EdgeAdj A, const double* __restrict__ x, double* __restrict__ part,
               BlockTab tab) {
  const Rows ch = rows_of(n, tab);
  double acc[1] = {0.0};
  for (long i = ch.lo + threadIdx.x; i < ch.hi; i += kBlock) {
    const double xi = x[i];
    if (cons_kind == 0) {
      acc[0] += xi * xi * xi * xi;
    } else {
      for (int k = A.urp[i]; k < A.urp[i + 1]; ++k) {
        const double p = xi * x[A.uci[k]];
        acc[0] += p * p;
      }
    }
  }
  block_sum_store<1>(acc, part + part_slot(tab));
}

// Fourth moments of q directions over the rows (DIAG family), for the block
// rank step: with the pairs (a <= b) numbered in row-major order and the
// pairs of pairs (P1 <= P2) likewise, entry e of block b is
//   part[b * ne + e] = sum over the block's rows i of V_ia V_ib V_ic V_id,
// ne = np (np + 1) / 2, np = q (q + 1) / 2.  V is n x q column-major.  The
// block's rows go through LDS kBlock at a time; thread t owns the entries
// t, t + kBlock, ... (at most kGramPerThread of them for q <= kMaxBlockDir).
constexpr int kMaxBlockDir = 8;
constexpr int kGramPerThread = 3;
__device__ __forceinline__ void pair_of(int pidx, int q, int& a, int& b) {
  a = 0;
  while (pidx >= q - a) {
    pidx -= q - a;
    ++a;
  }
  b = a + pidx;
}
__global__ void __launch_bounds__(kBlock)
k_gram4(long n, int q, const double* __restrict__ V, double* __restrict__ part) {
  __shared__ double tile[kBlock][kMaxBlockDir];
  const int np = q * (q + 1) / 2;
  const int ne = np * (np + 1) / 2;
  int ia[kGramPerThread], ib[kGramPerThread], ic[kGramPerThread], id[kGramPerThread];
  int cnt = 0;
  for (int e = threadIdx.x; e < ne && cnt < kGramPerThread; e += kBlock) {
    int p1 = 0, rem = e;
    while (rem >= np - p1) {
      rem -= np - p1;
      ++p1;
    }
    pair_of(p1, q, ia[cnt], ib[cnt]);
    pair_of(p1 + rem, q, ic[cnt], id[cnt]);
    ++cnt;
  }
  double acc[kGramPerThread] = {0.0, 0.0, 0.0};
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long lo = (long)blockIdx.x * per < n ? (long)blockIdx.x * per : n;
  const long hi = lo + per < n ? lo + per : n;
  for (long base = lo; base < hi; base += kBlock) {
    const long i = base + threadIdx.x;
    for (int k = 0; k < q; ++k) tile[threadIdx.x][k] = (i < hi) ? V[(long)k * n + i] : 0.0;
    __syncthreads();
    const int rows = hi - base < kBlock ? (int)(hi - base) : kBlock;
    for (int t = 0; t < cnt; ++t) {
      double s = 0.0;
      for (int rr = 0; rr < rows; ++rr) {
        const double* v = tile[rr];
        s += v[ia[t]] * v[ib[t]] * v[ic[t]] * v[id[t]];
      }
      acc[t] += s;
    }
    __syncthreads();
  }
  for (int t = 0; t < cnt; ++t) part[(long)blockIdx.x * ne + threadIdx.x + t * kBlock] = acc[t];
}

// The same moments for the edge rows of the trace + edge family: with
// K_e(ab) = (V_ia V_jb + V_ja V_ib) / 2 for edge e = (i, j) (the edge row of
// A(v_a v_b^T)), part[b * ne + e'] = sum over the block's edges of
// K_e(P1) K_e(P2) for the pair of pairs e' = (P1, P2).  Edges go through LDS
// kEdgeChunk at a time.
constexpr int kEdgeChunk = 128;
__global__ void __launch_bounds__(kBlock)
k_gram4_edges(long E, long n, int q, const int32_t* __restrict__ ei, const int32_t* __restrict__ ej,
              const double* __restrict__ V, double* __restrict__ part) {
  __shared__ double tile[kEdgeChunk][kMaxBlockDir * (kMaxBlockDir + 1) / 2];
  const int np = q * (q + 1) / 2;
  const int ne = np * (np + 1) / 2;
  int p1s[kGramPerThread], p2s[kGramPerThread];
  int cnt = 0;
  for (int e = threadIdx.x; e < ne && cnt < kGramPerThread; e += kBlock) {
    int p1 = 0, rem = e;
    while (rem >= np - p1) {
      rem -= np - p1;
      ++p1;
    }
    p1s[cnt] = p1;
    p2s[cnt] = p1 + rem;
    ++cnt;
  }
  double acc[kGramPerThread] = {0.0, 0.0, 0.0};
  const long per = (E + gridDim.x - 1) / gridDim.x;
  const long lo = (long)blockIdx.x * per < E ? (long)blockIdx.x * per : E;
  const long hi = lo + per < E ? lo + per : E;
  for (long base = lo; base < hi; base += kEdgeChunk) {
    const int rows = hi - base < kEdgeChunk ? (int)(hi - base) : kEdgeChunk;
    for (int idx = threadIdx.x; idx < rows * np; idx += kBlock) {
      const int el = idx / np, pp = idx % np;
      int a, b;
      pair_of(pp, q, a, b);
      const long i = ei[base + el], j = ej[base + el];
      tile[el][pp] = 0.5 * (V[(long)a * n + i] * V[(long)b * n + j] + V[(long)a * n + j] * V[(long)b * n + i]);
    }
    __syncthreads();
    for (int t = 0; t < cnt; ++t) {
      double s = 0.0;
      for (int rr = 0; rr < rows; ++rr) s += tile[rr][p1s[t]] * tile[rr][p2s[t]];
      acc[t] += s;
    }
    __syncthreads();
  }
  for (int t = 0; t < cnt; ++t) part[(long)blockIdx.x * ne + threadIdx.x + t * kBlock] = acc[t];
}

// ---- launchers (single instance: empty table, count 1, strides 0) ---------------

void launch_gram4_edges(long E, long n, int q, const int32_t* ei, const int32_t* ej, const double* V, double* part,
                        int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_gram4_edges, dim3(nb), dim3(kBlock), 0, st, E, n, q, ei, ej, V, part);
}

void launch_gram4(long n, int q, const double* V, double* part, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_gram4, dim3(nb), dim3(kBlock), 0, st, n, q, V, part);
}

int vec_blocks(long n) {
  long nb = (n + kBlock * 16 - 1) / (kBlock * 16);
  if (nb < 8) nb = 8;
  if (nb > 1024) nb = 1024;
  return (int)((nb + 7) / 8 * 8);
}

void launch_slack_mv(const Cost<double>& C, int cons_kind, const EdgeAdj& A, const double* y, double c_tr,
                     double j_coef, const DevScalars* sc, const double* x, double* out, hipStream_t st) {
  if (C.nh > 0) launch_hub_rows<double>(C, 1, 0, x, C.hsum, nullptr, 0, st);
  const long threads = C.n * kSpmvLpr;
  const int nb = (int)((threads + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_slack_mv, dim3(nb), dim3(kBlock), 0, st, C, cons_kind, A, y, c_tr, j_coef, sc, x, out);
}
void launch_slack_mv_tab(const Cost<double>& C, const double* y, const double* x, double* out, const BlockTab& tab,
                         int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_slack_mv_tab, dim3(nb), dim3(kBlock), 0, st, C, y, x, out, tab);
}
void launch_dots(long n, int ncol, const double* Q, long ldq, const double* w, double* part, int pstride, int nb,
                 double* h, hipStream_t st, const VecBatch& vb) {
  hipLaunchKernelGGL(k_dots, dim3(nb), dim3(kBlock), 0, st, n, ncol, Q, ldq, w, part, pstride, vb.tab);
  hipLaunchKernelGGL(k_fin_dots, dim3(ncol, vb.count), dim3(kBlock), 0, st, part, nb, pstride, ncol, h, vb.hstride,
                     vb.tab);
}
void launch_sub(long n, int ncol, const double* Q, long ldq, const double* h, double* w, double* part, int nb,
                hipStream_t st, const VecBatch& vb) {
  hipLaunchKernelGGL(k_sub, dim3(nb), dim3(kBlock), 0, st, n, ncol, Q, ldq, h, vb.hstride, w, part, vb.tab);
}
void launch_fin_ab(const double* part, int nb, const double* h1, const double* h2, int j, double* alpha, double* beta,
                   hipStream_t st, const VecBatch& vb) {
  hipLaunchKernelGGL(k_fin_ab, dim3(vb.count), dim3(kBlock), 0, st, part, nb, h1, h2, vb.hstride, j, alpha, beta,
                     vb.astride, vb.tab);
}
void launch_scale(long n, const double* w, const double* beta, double* q, double* part, int nb, double* qsum,
                  hipStream_t st, const VecBatch& vb, int bstride) {
  hipLaunchKernelGGL(k_scale, dim3(nb), dim3(kBlock), 0, st, n, w, beta, bstride, q, part, vb.tab);
  if (qsum) hipLaunchKernelGGL(k_fin_sum, dim3(vb.count), dim3(kBlock), 0, st, part, nb, qsum, 0, 0, vb.tab);
}
void launch_fin_sum(const double* part, int nb, double* out, int do_sqrt, hipStream_t st, const VecBatch& vb,
                    int ostride) {
  hipLaunchKernelGGL(k_fin_sum, dim3(vb.count), dim3(kBlock), 0, st, part, nb, out, ostride, do_sqrt, vb.tab);
}
void launch_mix(long n, double eps, const double* v, double* x, const double* norms, int nstride, double* part,
                int nb, hipStream_t st, const VecBatch& vb) {
  hipLaunchKernelGGL(k_mix, dim3(nb), dim3(kBlock), 0, st, n, eps, v, x, norms, nstride, part, vb.tab);
}
void launch_rand(long n, uint64_t seed, double* x, double* part, int nb, hipStream_t st, const VecBatch& vb) {
  hipLaunchKernelGGL(k_rand, dim3(nb), dim3(kBlock), 0, st, n, seed, x, part, vb.tab);
}
void launch_combine(long n, int ncol, const double* Q, long ldq, const double* s, double* v, double* part, int nb,
                    hipStream_t st, const VecBatch& vb, const int32_t* ncols) {
  hipLaunchKernelGGL(k_combine, dim3(nb), dim3(kBlock), 0, st, n, ncol, Q, ldq, s, vb.hstride, v, part, vb.tab,
                     ncols);
}
void launch_resid(long n, const double* z, const double* v, double theta, const double* thetas, double* part, int nb,
                  hipStream_t st, const VecBatch& vb) {
  hipLaunchKernelGGL(k_resid, dim3(nb), dim3(kBlock), 0, st, n, z, v, theta, thetas, part, vb.tab);
}
void launch_quartic_norm(long n, int cons_kind, const EdgeAdj& A, const double* x, double* part, int nb,
                         hipStream_t st, const VecBatch& vb) {
  hipLaunchKernelGGL(k_quartic_norm, dim3(nb), dim3(kBlock), 0, st, n, cons_kind, A, x, part, vb.tab);
}

// flags[q] = sc[q].flag, iters[q] = sc[q].iter (compact copy for the host).
__global__ void k_gather_flags(const DevScalars* __restrict__ sc, int count, int32_t* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  out[2 * q] = sc[q].flag;
  out[2 * q + 1] = sc[q].iter;
}

void launch_gather_flags(const DevScalars* sc, int count, int32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_flags, dim3((count + 63) / 64), dim3(64), 0, st, sc, count, out);
}

}  // namespace almbm
