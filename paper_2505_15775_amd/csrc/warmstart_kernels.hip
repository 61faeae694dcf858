// Learned warm start for the dual y0 of ALM-BM (MaxCut-type problems with the
// diagonal constraint family): per-vertex graph features, a small MLP
// (n_in -> h -> h -> 1, ReLU, FP32) forward and backward passes with
// deterministic gradient reductions, and the Adam update.  The MLP is a
// per-row dense product of width <= 64; at <= 64x64 weights per vertex it is
// bound by the vector ALUs and takes well under a millisecond per 10^7
// vertices, so plain FMA with weights staged in LDS is used.
#include "kernels.hpp"

namespace almbm {

constexpr int kWsFeat = 8;    // features per vertex
constexpr int kWsMaxH = 64;   // largest hidden width

// Feature pass 1: degree and weighted sums of a row of the cost.
//   f0 = log1p(deg_i), f1 = sum_j |S_ij|, f2 = sum_j S_ij, f3 = d_i,
//   f4 = d_i - sum_j |S_ij| (a Gershgorin bound: y_i <= it keeps Z(y) PSD).
// Pass 2 (neighbour statistics of log1p(deg)): f5 mean, f6 max, f7 mean of
// the neighbours' f1.
__global__ void __launch_bounds__(kBlock)
k_ws_feat1(Cost<double> C, float* __restrict__ F, float* __restrict__ deg_out) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= C.n) return;
  long k0 = 0, k1 = 0;
  if (C.ell > 0) {
    k0 = i * (long)C.ell;
    k1 = k0 + C.ell;
  } else if (C.rp) {
    k0 = C.rp[i];
    k1 = C.rp[i + 1];
  }
  double sa = 0.0, s = 0.0;
  int deg = 0;
  for (long k = k0; k < k1; ++k) {
    const double v = C.cv[k];
    if (v != 0.0 && C.ci[k] != i) {
      sa += fabs(v);
      s += v;
      ++deg;
    }
  }
  const double di = C.dg ? C.dg[i] : 0.0;
  float* f = F + i * kWsFeat;
  f[0] = log1pf((float)deg);
  f[1] = (float)sa;
  f[2] = (float)s;
  f[3] = (float)di;
  f[4] = (float)(di - sa);
  deg_out[i] = f[0];
}

__global__ void __launch_bounds__(kBlock)
k_ws_feat2(Cost<double> C, const float* __restrict__ ldeg, float* __restrict__ F) {
  const long i = (long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= C.n) return;
  long k0 = 0, k1 = 0;
  if (C.ell > 0) {
    k0 = i * (long)C.ell;
    k1 = k0 + C.ell;
  } else if (C.rp) {
    k0 = C.rp[i];
    k1 = C.rp[i + 1];
  }
  float sum = 0.f, mx = 0.f, s1 = 0.f;
  int cnt = 0;
  for (long k = k0; k < k1; ++k) {
    const int j = C.ci[k];
    if (C.cv[k] == 0.0 || j == i) continue;
    const float d = ldeg[j];
    sum += d;
    mx = fmaxf(mx, d);
    s1 += F[(long)j * kWsFeat + 1];
    ++cnt;
  }
  float* f = F + i * kWsFeat;
  const float inv = cnt ? 1.f / (float)cnt : 0.f;
  f[5] = sum * inv;
  f[6] = mx;
  f[7] = s1 * inv;
}

// Parameter layout (floats): W1[nin][h], b1[h], W2[h][h], b2[h], W3[h], b3[1].
__device__ __forceinline__ int ws_nparams(int nin, int h) { return nin * h + h + h * h + h + h + 1; }

// Stage the parameters in LDS (<= 8*64 + 64 + 64*64 + 64 + 64 + 1 floats).
__device__ __forceinline__ void ws_load_params(const float* __restrict__ P, float* __restrict__ S, int np) {
  for (int k = threadIdx.x; k < np; k += kBlock) S[k] = P[k];
  __syncthreads();
}

// One vertex: hidden activations a1, a2 (pre-ReLU kept for the backward pass).
template <int H>
__device__ __forceinline__ float ws_forward_row(const float* __restrict__ S, int nin, const float* __restrict__ x,
                                                float (&z1)[H], float (&z2)[H]) {
  const float* W1 = S;
  const float* b1 = W1 + nin * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float b3 = W3[H];
#pragma unroll
  for (int o = 0; o < H; ++o) z1[o] = b1[o];
  for (int i = 0; i < nin; ++i) {
    const float xi = x[i];
#pragma unroll
    for (int o = 0; o < H; ++o) z1[o] += xi * W1[i * H + o];
  }
#pragma unroll
  for (int o = 0; o < H; ++o) z2[o] = b2[o];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float a = fmaxf(z1[i], 0.f);
#pragma unroll
    for (int o = 0; o < H; ++o) z2[o] += a * W2[i * H + o];
  }
  float out = b3;
#pragma unroll
  for (int o = 0; o < H; ++o) out += fmaxf(z2[o], 0.f) * W3[o];
  return out;
}

template <int H>
__global__ void __launch_bounds__(kBlock)
k_ws_forward(const float* __restrict__ P, int nin, const float* __restrict__ mu, const float* __restrict__ isd,
             long n, const float* __restrict__ X, double* __restrict__ out) {
  __shared__ float S[kWsFeat * kWsMaxH + kWsMaxH + kWsMaxH * kWsMaxH + kWsMaxH + kWsMaxH + 1];
  ws_load_params(P, S, ws_nparams(nin, H));
  const long stride = (long)gridDim.x * kBlock;
  for (long v = (long)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
    float z1[H], z2[H], x[kWsFeat];
#pragma unroll
    for (int i = 0; i < kWsFeat; ++i) x[i] = i < nin ? (X[v * nin + i] - mu[i]) * isd[i] : 0.f;
    out[v] = (double)ws_forward_row<H>(S, nin, x, z1, z2);
  }
}

// Column means of an n x 8 feature array (fixed-order two-level reduction).
__global__ void __launch_bounds__(kBlock)
k_ws_pool(const float* __restrict__ F, long n, double* __restrict__ part) {
  double acc[kWsFeat];
#pragma unroll
  for (int k = 0; k < kWsFeat; ++k) acc[k] = 0.0;
  const long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long lo = (long)blockIdx.x * chunk;
  const long hi = lo + chunk < n ? lo + chunk : n;
  for (long v = lo + threadIdx.x; v < hi; v += kBlock)
#pragma unroll
    for (int k = 0; k < kWsFeat; ++k) acc[k] += F[v * kWsFeat + k];
  block_sum_store<kWsFeat>(acc, part + (long)blockIdx.x * kWsFeat);
}

__global__ void __launch_bounds__(kBlock)
k_ws_pool_fin(const double* __restrict__ part, int nb, long n, double* __restrict__ out) {
  if (threadIdx.x < kWsFeat) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[(long)b * kWsFeat + threadIdx.x];
    out[threadIdx.x] = n > 0 ? t / (double)n : 0.0;
  }
}

// Forward + backward of the mean squared error (1/n) sum_v (f(x_v) - t_v)^2.
// A block owns a contiguous range of vertices and walks it 256 rows at a time:
// every thread computes one row's activations and deltas, then the rows are
// staged in LDS one wave (64 rows) at a time and each thread adds, in row
// order, the contributions to the parameter gradients it owns (k = tid,
// tid + 256, ...).  Per-block partials are reduced later in block order, so the
// gradient is deterministic.
constexpr int kWsRows = 64;

template <int H>
__global__ void __launch_bounds__(kBlock)
k_ws_backward(const float* __restrict__ P, int nin, const float* __restrict__ mu, const float* __restrict__ isd, long n,
              const float* __restrict__ X, const float* __restrict__ T, float inv_n, float* __restrict__ gpart,
              double* __restrict__ lpart) {
  __shared__ float S[kWsFeat * kWsMaxH + kWsMaxH + kWsMaxH * kWsMaxH + kWsMaxH + kWsMaxH + 1];
  __shared__ float sX[kWsRows][kWsFeat];
  __shared__ float sA1[kWsRows][H];
  __shared__ float sD1[kWsRows][H];
  __shared__ float sA2[kWsRows][H];
  __shared__ float sD2[kWsRows][H];
  __shared__ float sDo[kWsRows];
  __shared__ double lred[kBlock / kWave];
  const int np = ws_nparams(nin, H);
  ws_load_params(P, S, np);
  const float* W2 = S + nin * H + H;
  const float* W3 = W2 + H * H + H;
  constexpr int KMAX = (kWsFeat * kWsMaxH + kWsMaxH + kWsMaxH * kWsMaxH + kWsMaxH + kWsMaxH + 1 + kBlock - 1) / kBlock;
  float gacc[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) gacc[j] = 0.f;
  const int oW1 = 0, ob1 = nin * H, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + H;
  const long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long lo = (long)blockIdx.x * chunk;
  const long hi = lo + chunk < n ? lo + chunk : n;
  double loss = 0.0;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  for (long base = lo; base < hi; base += kBlock) {
    const long v = base + threadIdx.x;
    const bool act = v < hi;
    float z1[H], z2[H], d2[H], d1[H];
    float dout = 0.f;
    float x[kWsFeat];
#pragma unroll
    for (int i = 0; i < kWsFeat; ++i) x[i] = (act && i < nin) ? (X[v * nin + i] - mu[i]) * isd[i] : 0.f;
    if (act) {
      const float y = ws_forward_row<H>(S, nin, x, z1, z2);
      const float e = y - T[v];
      loss += (double)e * (double)e;
      dout = 2.f * e * inv_n;
    } else {
#pragma unroll
      for (int o = 0; o < H; ++o) z1[o] = z2[o] = 0.f;
    }
#pragma unroll
    for (int o = 0; o < H; ++o) d2[o] = (z2[o] > 0.f) ? dout * W3[o] : 0.f;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      float a = 0.f;
#pragma unroll
      for (int o = 0; o < H; ++o) a += W2[i * H + o] * d2[o];
      d1[i] = (z1[i] > 0.f) ? a : 0.f;
    }
    for (int w = 0; w < kBlock / kWave; ++w) {
      __syncthreads();
      if (wave == w) {
#pragma unroll
        for (int i = 0; i < kWsFeat; ++i) sX[lane][i] = x[i];
#pragma unroll
        for (int o = 0; o < H; ++o) {
          sA1[lane][o] = fmaxf(z1[o], 0.f);
          sD1[lane][o] = d1[o];
          sA2[lane][o] = fmaxf(z2[o], 0.f);
          sD2[lane][o] = d2[o];
        }
        sDo[lane] = dout;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        const int k = threadIdx.x + j * kBlock;
        if (k >= np) break;
        float a = 0.f;
        if (k < ob1) {
          const int i = (k - oW1) / H, o = (k - oW1) % H;
          for (int rr = 0; rr < kWsRows; ++rr) a += sX[rr][i] * sD1[rr][o];
        } else if (k < oW2) {
          const int o = k - ob1;
          for (int rr = 0; rr < kWsRows; ++rr) a += sD1[rr][o];
        } else if (k < ob2) {
          const int i = (k - oW2) / H, o = (k - oW2) % H;
          for (int rr = 0; rr < kWsRows; ++rr) a += sA1[rr][i] * sD2[rr][o];
        } else if (k < oW3) {
          const int o = k - ob2;
          for (int rr = 0; rr < kWsRows; ++rr) a += sD2[rr][o];
        } else if (k < ob3) {
          const int o = k - oW3;
          for (int rr = 0; rr < kWsRows; ++rr) a += sA2[rr][o] * sDo[rr];
        } else {
          for (int rr = 0; rr < kWsRows; ++rr) a += sDo[rr];
        }
        gacc[j] += a;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    const int k = threadIdx.x + j * kBlock;
    if (k < np) gpart[(long)blockIdx.x * np + k] = gacc[j];
  }
  loss = wave_sum(loss);
  if (threadIdx.x % kWave == 0) lred[threadIdx.x / kWave] = loss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += lred[w];
    lpart[blockIdx.x] = t;
  }
}

// grad[k] = sum over blocks of gpart[b][k] (block order); loss = (1/n) sum of
// the per-block squared errors, same order.
__global__ void __launch_bounds__(kBlock)
k_ws_reduce(const float* __restrict__ gpart, const double* __restrict__ lpart, int nb, int np, double inv_n,
            float* __restrict__ grad, double* __restrict__ loss_out) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < np) {
    float a = 0.f;
    for (int b = 0; b < nb; ++b) a += gpart[(long)b * np + k];
    grad[k] = a;
  }
  if (k == 0 && loss_out) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += lpart[b];
    *loss_out = t * inv_n;
  }
}

// Adam (Kingma & Ba, 2015), bias-corrected.
__global__ void __launch_bounds__(kBlock)
k_ws_adam(float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v, int np,
          float lr, float b1, float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= np) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  P[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// ---- launchers -------------------------------------------------------------------

void launch_ws_features(const Cost<double>& C, float* F, float* ldeg, hipStream_t st) {
  const int nb = (int)((C.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_ws_feat1, dim3(nb), dim3(kBlock), 0, st, C, F, ldeg);
  hipLaunchKernelGGL(k_ws_feat2, dim3(nb), dim3(kBlock), 0, st, C, ldeg, F);
}

int ws_param_count(int nin, int h) { return nin * h + h + h * h + h + h + 1; }

bool launch_ws_forward(const float* P, int nin, int h, const float* mu, const float* isd, long n, const float* X,
                       double* out, hipStream_t st) {
  long nb = (n + kBlock - 1) / kBlock;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  if (h == 16) hipLaunchKernelGGL(k_ws_forward<16>, dim3(nb), dim3(kBlock), 0, st, P, nin, mu, isd, n, X, out);
  else if (h == 32) hipLaunchKernelGGL(k_ws_forward<32>, dim3(nb), dim3(kBlock), 0, st, P, nin, mu, isd, n, X, out);
  else if (h == 64) hipLaunchKernelGGL(k_ws_forward<64>, dim3(nb), dim3(kBlock), 0, st, P, nin, mu, isd, n, X, out);
  else return false;
  return true;
}

void launch_ws_pool(const float* F, long n, double* part, int nb, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_ws_pool, dim3(nb), dim3(kBlock), 0, st, F, n, part);
  hipLaunchKernelGGL(k_ws_pool_fin, dim3(1), dim3(kBlock), 0, st, part, nb, n, out);
}

bool launch_ws_backward(const float* P, int nin, int h, const float* mu, const float* isd, long n, const float* X,
                        const float* T, float* gpart, double* lpart, int nb, float* grad, double* loss,
                        hipStream_t st) {
  const float inv_n = n > 0 ? 1.f / (float)n : 0.f;
  if (h == 16)
    hipLaunchKernelGGL(k_ws_backward<16>, dim3(nb), dim3(kBlock), 0, st, P, nin, mu, isd, n, X, T, inv_n, gpart,
                       lpart);
  else if (h == 32)
    hipLaunchKernelGGL(k_ws_backward<32>, dim3(nb), dim3(kBlock), 0, st, P, nin, mu, isd, n, X, T, inv_n, gpart,
                       lpart);
  else if (h == 64)
    hipLaunchKernelGGL(k_ws_backward<64>, dim3(nb), dim3(kBlock), 0, st, P, nin, mu, isd, n, X, T, inv_n, gpart,
                       lpart);
  else
    return false;
  const int np = ws_param_count(nin, h);
  hipLaunchKernelGGL(k_ws_reduce, dim3((np + kBlock - 1) / kBlock), dim3(kBlock), 0, st, gpart, lpart, nb, np,
                     n > 0 ? 1.0 / (double)n : 0.0, grad, loss);
  return true;
}

void launch_ws_adam(float* P, const float* g, float* m, float* v, int np, float lr, float b1, float b2, float eps,
                    int step, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_ws_adam, dim3((np + kBlock - 1) / kBlock), dim3(kBlock), 0, st, P, g, m, v, np, lr, b1, b2,
                     eps, c1, c2);
}

}  // namespace almbm
