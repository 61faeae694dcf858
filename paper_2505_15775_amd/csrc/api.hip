// C ABI of libalmbm: handle, workspace, entry points and the host side of the
// ALM-BM solve (Alg. 1 of arxiv 2505.15775 with p = 1 rank adaptation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "alm_bm.h"
#include "api_internal.hpp"
#include "launch.hpp"

using namespace almbm;

// --------------------------------------------------------------------- errors

static thread_local std::string g_err;

static alm_bm_status fail(alm_bm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

alm_bm_status almbm::set_error(alm_bm_status s, const std::string& msg) { return fail(s, msg); }

#define HIPCHK(x)                                                                                         \
  do {                                                                                                    \
    hipError_t e_ = (x);                                                                                  \
    if (e_ != hipSuccess) return fail(ALM_BM_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));   \
  } while (0)

#define STCHK(x)                       \
  do {                                 \
    alm_bm_status s_ = (x);            \
    if (s_ < 0) return s_;             \
  } while (0)

// --------------------------------------------------------------------- handle

constexpr int kMaxBlockDirHost = 8;  // largest rank_block (directions of a block rank step)

struct alm_bm_problem {
  alm_bm_problem_desc d{};
  double cnorm = 0.0;  // ||C||_F
  double bnorm = 0.0;  // ||b||_2
  Cost<double> C64{};
  Cost<float> C32{};
  EdgeAdj adj{};
  double* wE = nullptr;
  int nblk = 0;
  int max_blocks = 0;
  int variant = 0;
  BlockTab tab{};                 // batched super-problem: per-block instance rows
  int count = 1;                  // instances (DevScalars in sc_solve)
  double rho = 1.0;               // edge rows' penalty / sigma (set for the length of a solve)
  double* part = nullptr;     // nblk * (NUM_P + kMaxR)
  double* part2 = nullptr;    // edge family: 64 * (NUM_P + kMaxR), first stage of the finalizers
  double* part_c2 = nullptr;  // nblk
  double* part_vec = nullptr; // vec kernels
  DevScalars* sc_api = nullptr;
  DevScalars* sc_solve = nullptr;
  DevScalars* sc_host = nullptr;  // pinned mirror
  void* G = nullptr;              // n * r_max storage
  void* Rtmp = nullptr;           // n * r_max storage
  void* Qbuf = nullptr;           // n * r_max arithmetic type: C G of the inner loop
  int ladder_r = 0;               // rank of the float factor in R32 after a promoted solve (0: none)
  void* R32 = nullptr;            // float factor, gradient and relayout scratch for
  void* G32 = nullptr;            //   the BF16 -> float precision ladder
  void* Rt32 = nullptr;
  hipStream_t ss = nullptr;       // solve stream (non-blocking, default priority)
  double* Av = nullptr;           // m
  double* ybuf = nullptr;         // m
  // Lanczos workspace
  int kmax = 0;
  int lnb = 0;
  double* Q = nullptr;
  double* lw = nullptr;
  double* lh1 = nullptr;
  double* lh2 = nullptr;
  double* lalpha = nullptr;
  double* lbeta = nullptr;
  double* lpart = nullptr;
  double* lpart2 = nullptr;
  double* lv = nullptr;
  double* ls = nullptr;
  double* lscal = nullptr;
  std::vector<void*> allocs;
  double* bk_h = nullptr;         // block Krylov: (kmax+1)^2 projected matrix, column sums, Ritz coefficients
  double* bk_colsum = nullptr;
  double* bk_coef = nullptr;
  double* vblk = nullptr;         // block rank step: n x rank_block_max directions, their coefficients,
  double* ycoef = nullptr;        //   fourth-moment partials (reserved at create)
  double* gpart = nullptr;
  int32_t* hub_list = nullptr;    // hub rows: capacity hub_cap rows, sums 2 x hub_cap x r_max per precision
  double* hub_sum64 = nullptr;
  float* hub_sum32 = nullptr;
  long hub_cap = 0;
  LbfgsState* lbs = nullptr;      // L-BFGS state and rings (lbfgs_memory_max + 1 slots each)
  void* lb_e = nullptr;
  void* lb_y = nullptr;
  long lb_stride = 0;             // elements per ring slot
  int lb_m = 0;                   // memory of the running solve (0: gradient descent)
};

// Rings of storage type S (RingT of the factor's type) while an L-BFGS solve
// runs; empty otherwise.
template <typename S> static LbfgsRing<S> lbfgs_ring(const alm_bm_problem* p) {
  if (p->lb_m <= 0) return LbfgsRing<S>{};
  return LbfgsRing<S>{p->lbs, static_cast<S*>(p->lb_e), static_cast<S*>(p->lb_y), p->lb_stride};
}

static size_t esize(alm_bm_precision p) { return p == ALM_BM_F64 ? 8 : (p == ALM_BM_F32 ? 4 : 2); }

static alm_bm_status dalloc(alm_bm_problem* p, void** out, size_t bytes) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) return fail(ALM_BM_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  p->allocs.push_back(*out);
  return ALM_BM_OK;
}
template <typename X>
static alm_bm_status dalloc_t(alm_bm_problem* p, X** out, size_t count) {
  void* v = nullptr;
  STCHK(dalloc(p, &v, count * sizeof(X)));
  *out = static_cast<X*>(v);
  return ALM_BM_OK;
}

static void free_all(alm_bm_problem* p) {
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
  if (p->ss) (void)hipStreamDestroy(p->ss);
  p->ss = nullptr;
  if (p->sc_host) (void)hipHostFree(p->sc_host);
  p->sc_host = nullptr;
}

template <typename T> static const Cost<typename Acc<T>::type>& cost_of(const alm_bm_problem* p);
template <> const Cost<double>& cost_of<double>(const alm_bm_problem* p) { return p->C64; }
template <> const Cost<float>& cost_of<float>(const alm_bm_problem* p) { return p->C32; }
template <> const Cost<float>& cost_of<bf16>(const alm_bm_problem* p) { return p->C32; }

// Rows of the cost with more stored entries than this are hub rows (Cost):
// twice the average row length (rounded up), at least 32.  On R-MAT graphs of
// 2^20 and 2^22 vertices this was within a few per cent of the best
// threshold of a sweep from 16 to 256 entries; Poisson-degree graphs get none.
static int32_t hub_threshold(long nnz, long n) {
  const long avg = (nnz + n - 1) / std::max<long>(1, n);
  return (int32_t)std::min<long>(INT32_MAX, std::max<long>(32, 2 * avg));
}

// Hub rows of a DIAG-family CSR cost.  min_degree < 0: none; 0: the default
// threshold; > 0: rows with more than min_degree entries.  reserve: allocate
// the hub list and sums for exactly this many hubs (alm_bm_create); otherwise
// the hubs must fit the capacity reserved then, and the arrays are rewritten
// in place after a device synchronisation (no allocation).
static alm_bm_status build_hubs(alm_bm_problem* p, int32_t min_degree, bool reserve) {
  const auto& d = p->d;
  for (auto* c : {&p->C64.nh, &p->C32.nh}) *c = 0;
  if (d.cons_kind != ALM_BM_CONS_DIAG || d.ell_width != 0 || d.nnz == 0 || min_degree < 0) return ALM_BM_OK;
  const long n = d.n;
  std::vector<int32_t> hrp(n + 1);
  HIPCHK(hipMemcpy(hrp.data(), d.row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  const int32_t thr = min_degree == 0 ? hub_threshold(d.nnz, n) : min_degree;
  std::vector<int32_t> hubs;
  for (long i = 0; i < n; ++i)
    if (hrp[i + 1] - hrp[i] > thr) hubs.push_back((int32_t)i);
  const long nh = (long)hubs.size();
  if (reserve) {
    p->hub_cap = nh;
    if (nh == 0) return ALM_BM_OK;
    STCHK(dalloc_t(p, &p->hub_list, nh));
    STCHK(dalloc_t(p, &p->hub_sum64, 2 * nh * d.r_max));
    if (d.precision != ALM_BM_F64) STCHK(dalloc_t(p, &p->hub_sum32, 2 * nh * d.r_max));
  } else if (nh > p->hub_cap) {
    return fail(ALM_BM_ERR_INVALID_ARG, "set_hub_threshold: " + std::to_string(nh) + " hub rows at threshold " +
                                            std::to_string(thr) + ", the handle reserved " +
                                            std::to_string(p->hub_cap) + " (desc.hub_min_degree)");
  } else {
    HIPCHK(hipDeviceSynchronize());  // earlier launches may still read the list
  }
  if (nh == 0) return ALM_BM_OK;
  HIPCHK(hipMemcpy(p->hub_list, hubs.data(), nh * sizeof(int32_t), hipMemcpyHostToDevice));
  p->C64.hthr = thr;
  p->C64.hrow = p->hub_list;
  p->C64.hsum = p->hub_sum64;
  p->C64.hsum2 = p->hub_sum64 + nh * d.r_max;
  p->C64.nh = (int32_t)nh;
  if (d.precision != ALM_BM_F64) {
    p->C32.hthr = thr;
    p->C32.hrow = p->hub_list;
    p->C32.hsum = p->hub_sum32;
    p->C32.hsum2 = p->hub_sum32 + nh * d.r_max;
    p->C32.nh = (int32_t)nh;
  }
  return ALM_BM_OK;
}

// Run f.template operator()<T>() for the storage type of precision `prec`.
template <typename F>
static auto with_storage(alm_bm_precision prec, F&& f) {
  if (prec == ALM_BM_F64) return f.template operator()<double>();
  if (prec == ALM_BM_F32) return f.template operator()<float>();
  return f.template operator()<bf16>();
}

// --------------------------------------------------------------------- host helpers

static bool check_csr(const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, long n, long nnz,
                      std::string& why) {
  if (rp[0] != 0 || rp[n] != nnz) {
    why = "row_ptr[0] must be 0 and row_ptr[n] must equal nnz";
    return false;
  }
  for (long i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) {
      why = "row_ptr not monotone at row " + std::to_string(i);
      return false;
    }
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      if (ci[k] < 0 || ci[k] >= n) {
        why = "col_idx out of range at entry " + std::to_string(k);
        return false;
      }
      if (k > rp[i] && ci[k] < ci[k - 1]) {
        why = "col_idx not ascending in row " + std::to_string(i);
        return false;
      }
    }
  }
  return true;
}

extern "C" alm_bm_status alm_bm_maxcut_cost_host(int64_t n, int64_t m_edges, const int32_t* ei, const int32_t* ej,
                                                 const double* w, int32_t* row_ptr, int32_t* col_idx, double* val,
                                                 double* diag, int64_t* nnz_out) {
  if (n <= 0 || m_edges < 0 || (m_edges > 0 && (!ei || !ej || !w)) || !row_ptr || !diag || !nnz_out)
    return fail(ALM_BM_ERR_INVALID_ARG, "maxcut_cost_host: bad arguments");
  if (2 * m_edges > INT32_MAX) return fail(ALM_BM_ERR_UNSUPPORTED, "maxcut_cost_host: more than 2^31 entries");
  std::vector<int64_t> cnt(n + 1, 0);
  for (int64_t e = 0; e < m_edges; ++e) {
    const int32_t i = ei[e], j = ej[e];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j)
      return fail(ALM_BM_ERR_INVALID_PATTERN, "maxcut_cost_host: edge " + std::to_string(e) + " invalid");
    cnt[i + 1]++;
    cnt[j + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int64_t> cur(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < n; ++i) diag[i] = 0.0;
  // lower entries (row = larger endpoint) first, then upper: ascending columns
  // within each row when the edge list is sorted by (min, max)
  for (int64_t e = 0; e < m_edges; ++e) {
    const int32_t i = std::min(ei[e], ej[e]), j = std::max(ei[e], ej[e]);
    col_idx[cur[j]] = i;
    val[cur[j]++] = 0.25 * w[e];
  }
  for (int64_t e = 0; e < m_edges; ++e) {
    const int32_t i = std::min(ei[e], ej[e]), j = std::max(ei[e], ej[e]);
    col_idx[cur[i]] = j;
    val[cur[i]++] = 0.25 * w[e];
    diag[i] -= 0.25 * w[e];
    diag[j] -= 0.25 * w[e];
  }
  // sort rows that are not ascending, merge duplicates, compact
  int64_t out = 0;
  std::vector<std::pair<int32_t, double>> tmp;
  row_ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t a = cnt[i], b = cnt[i + 1];
    bool sorted = true;
    for (int64_t k = a + 1; k < b; ++k)
      if (col_idx[k] <= col_idx[k - 1]) {
        sorted = false;
        break;
      }
    if (!sorted) {
      tmp.clear();
      for (int64_t k = a; k < b; ++k) tmp.emplace_back(col_idx[k], val[k]);
      std::sort(tmp.begin(), tmp.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
      int64_t k = a;
      for (size_t t = 0; t < tmp.size(); ++t) {
        col_idx[k] = tmp[t].first;
        val[k] = tmp[t].second;
        ++k;
      }
    }
    for (int64_t k = a; k < b; ++k) {
      if (out > row_ptr[i] && col_idx[out - 1] == col_idx[k]) {
        val[out - 1] += val[k];
      } else {
        col_idx[out] = col_idx[k];
        val[out] = val[k];
        ++out;
      }
    }
    row_ptr[i + 1] = (int32_t)out;
  }
  *nnz_out = out;
  return ALM_BM_OK;
}

extern "C" void alm_bm_default_options(alm_bm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps_kkt = 1e-6;
  o->sigma = 1.0;
  o->max_outer = 1000;
  o->max_inner = 500;
  o->step_rule = ALM_BM_STEP_EXACT;
  o->eta_fixed = 1e-3;
  o->rank_policy = ALM_BM_RANK_ADAPT;
  o->r_cap = 0;
  o->tau_rank = 0.0;
  o->expand_needs_inner = 0;
  o->inner_tol_scale = 0.1;
  o->inner_tol_decay = 0.7;
  o->lanczos_kmax = 0;
  o->lanczos_tol_rel = 0.1;
  o->seed = 1;
  o->graph_unroll = 8;
  o->verbose = 0;
  o->time_limit_s = 0.0;
  o->bf16_promote = 1;
  o->refresh_every = 0;
  o->lanczos_restarts = 3;
  o->sigma_edges = 0.0;
  o->sigma_growth = 1.0;
  o->sigma_max = 1e6;
  o->pinf_reduction = 0.25;
  o->rank_block = 1;
  o->inner_solver = ALM_BM_INNER_GD;
  o->lbfgs_memory = 3;
}

extern "C" const char* alm_bm_last_error(void) { return g_err.c_str(); }

extern "C" void alm_bm_abi_sizes(int64_t* out) {
  if (!out) return;
  out[0] = (int64_t)sizeof(alm_bm_problem_desc);
  out[1] = (int64_t)sizeof(alm_bm_options);
  out[2] = (int64_t)sizeof(alm_bm_result);
}

// --------------------------------------------------------------------- create / destroy

int almbm::row_blocks(long n) {
  long nb = (n + 63) / 64;
  if (nb < 8) nb = 8;
  if (nb > 4096) nb = 4096;
  return (int)((nb + 7) / 8 * 8);
}

// Largest grid a handle supports (blocks of fewer than 8 rows are pointless).
static int max_row_blocks(long n) {
  long nb = (n + 7) / 8;
  if (nb < 8) nb = 8;
  if (nb > 16384) nb = 16384;
  return (int)((nb + 7) / 8 * 8);
}

extern "C" alm_bm_status alm_bm_create(const alm_bm_problem_desc* desc, hipStream_t st, alm_bm_problem** out) {
  if (!desc || !out) return fail(ALM_BM_ERR_INVALID_ARG, "create: null desc or out");
  *out = nullptr;
  const alm_bm_problem_desc& d = *desc;
  if (d.n <= 0 || d.n > INT32_MAX) return fail(ALM_BM_ERR_INVALID_ARG, "create: n out of range");
  if (d.r_max < 1 || d.r_max > kMaxR) return fail(ALM_BM_ERR_INVALID_ARG, "create: r_max must be in 1..128");
  if (d.lanczos_kmax < 0 || d.lanczos_kmax > 512)
    return fail(ALM_BM_ERR_INVALID_ARG, "create: lanczos_kmax must be in 0..512");
  if (d.rank_block_max < 0 || d.rank_block_max > kMaxBlockDirHost)
    return fail(ALM_BM_ERR_INVALID_ARG, "create: rank_block_max must be in 0..8");
  if (d.lbfgs_memory_max < 0 || d.lbfgs_memory_max > kMaxLbfgs)
    return fail(ALM_BM_ERR_INVALID_ARG, "create: lbfgs_memory_max must be in 0..8");
  if (d.lbfgs_memory_max > 0 && d.cons_kind != ALM_BM_CONS_DIAG)
    return fail(ALM_BM_ERR_UNSUPPORTED, "create: the L-BFGS inner solver is for the DIAG family");
  if (d.precision != ALM_BM_F64 && d.precision != ALM_BM_F32 && d.precision != ALM_BM_BF16)
    return fail(ALM_BM_ERR_INVALID_ARG, "create: unknown precision");
  if (!d.b) return fail(ALM_BM_ERR_INVALID_ARG, "create: b is null");
  if (d.nnz < 0 || (d.nnz > 0 && (!d.col_idx || !d.val)))
    return fail(ALM_BM_ERR_INVALID_ARG, "create: nnz > 0 needs col_idx and val");
  if (d.nnz > INT32_MAX) return fail(ALM_BM_ERR_UNSUPPORTED, "create: nnz >= 2^31 needs 64-bit indices");
  if (d.ell_width < 0) return fail(ALM_BM_ERR_INVALID_ARG, "create: ell_width < 0");
  if (d.ell_width > 0 && d.nnz != d.n * (int64_t)d.ell_width)
    return fail(ALM_BM_ERR_INVALID_ARG, "create: ELL needs nnz = n * ell_width");
  if (d.ell_width == 0 && d.nnz > 0 && !d.row_ptr) return fail(ALM_BM_ERR_INVALID_ARG, "create: CSR needs row_ptr");
  if (d.cons_kind == ALM_BM_CONS_DIAG) {
    if (d.m != d.n) return fail(ALM_BM_ERR_INVALID_ARG, "create: DIAG needs m = n");
    if (d.j_coef != 0.0) return fail(ALM_BM_ERR_UNSUPPORTED, "create: DIAG constraints with a -J cost term");
  } else if (d.cons_kind == ALM_BM_CONS_TRACE_EDGES) {
    if (d.n_edges < 0 || d.m != d.n_edges + 1) return fail(ALM_BM_ERR_INVALID_ARG, "create: TRACE_EDGES needs m = n_edges + 1");
    if (d.n_edges > 0 && (!d.edge_i || !d.edge_j)) return fail(ALM_BM_ERR_INVALID_ARG, "create: edge arrays null");
    if (2 * d.n_edges > INT32_MAX) return fail(ALM_BM_ERR_UNSUPPORTED, "create: too many edges");
  } else {
    return fail(ALM_BM_ERR_INVALID_ARG, "create: unknown constraint kind");
  }
  HIPCHK(hipStreamSynchronize(st));

  alm_bm_problem* p = new alm_bm_problem();
  p->d = d;
  const long n = d.n;
  auto bail = [&](alm_bm_status s) {
    free_all(p);
    delete p;
    return s;
  };
#define CK(x)                          \
  do {                                 \
    alm_bm_status s_ = (x);            \
    if (s_ < 0) return bail(s_);       \
  } while (0)
#define HK(x)                                                                                          \
  do {                                                                                                 \
    hipError_t e_ = (x);                                                                               \
    if (e_ != hipSuccess) return bail(fail(ALM_BM_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_))); \
  } while (0)

  // ---- host copies for validation, norms and the edge adjacency
  std::vector<double> hval(d.nnz), hdg(d.diag ? n : 0), hb(d.m);
  if (d.nnz) HK(hipMemcpy(hval.data(), d.val, d.nnz * sizeof(double), hipMemcpyDeviceToHost));
  if (d.diag) HK(hipMemcpy(hdg.data(), d.diag, n * sizeof(double), hipMemcpyDeviceToHost));
  HK(hipMemcpy(hb.data(), d.b, d.m * sizeof(double), hipMemcpyDeviceToHost));
  if (d.validate && d.nnz) {
    std::vector<int32_t> hci(d.nnz);
    HK(hipMemcpy(hci.data(), d.col_idx, d.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (d.ell_width > 0) {
      for (long k = 0; k < d.nnz; ++k)
        if (hci[k] < 0 || hci[k] >= n) return bail(fail(ALM_BM_ERR_INVALID_PATTERN, "ELL col_idx out of range"));
    } else {
      std::vector<int32_t> hrp(n + 1);
      HK(hipMemcpy(hrp.data(), d.row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
      std::string why;
      if (!check_csr(hrp, hci, n, d.nnz, why)) return bail(fail(ALM_BM_ERR_INVALID_PATTERN, "CSR: " + why));
    }
  }
  for (double v : hval)
    if (!std::isfinite(v)) return bail(fail(ALM_BM_ERR_NUMERIC, "create: non-finite cost value"));
  for (double v : hb)
    if (!std::isfinite(v)) return bail(fail(ALM_BM_ERR_NUMERIC, "create: non-finite b"));
  // ||S + D - jJ||_F^2 = ||S + D||^2 - 2 j sum(S + D) + j^2 n^2
  {
    double s2 = 0.0, s1 = 0.0;
    for (double v : hval) {
      s2 += v * v;
      s1 += v;
    }
    for (double v : hdg) {
      s2 += v * v;
      s1 += v;
    }
    const double j = d.j_coef;
    p->cnorm = std::sqrt(std::max(0.0, s2 - 2.0 * j * s1 + j * j * (double)n * (double)n));
    double b2 = 0.0;
    for (double v : hb) b2 += v * v;
    p->bnorm = std::sqrt(b2);
  }
  p->C64 = Cost<double>{n, d.ell_width > 0 ? nullptr : (d.nnz ? d.row_ptr : nullptr), d.col_idx, d.val, d.ell_width,
                        d.diag};
  if (d.nnz == 0) p->C64.rp = nullptr, p->C64.ell = 0;

  // ---- float copies of the cost for the F32 / BF16 modes
  if (d.precision != ALM_BM_F64) {
    float* cv32 = nullptr;
    float* dg32 = nullptr;
    if (d.nnz) {
      CK(dalloc_t(p, &cv32, d.nnz));
      launch_convert<double, float>(d.nnz, d.val, cv32, st);
    }
    if (d.diag) {
      CK(dalloc_t(p, &dg32, n));
      launch_convert<double, float>(n, d.diag, dg32, st);
    }
    p->C32 = Cost<float>{n, p->C64.rp, d.col_idx, cv32, p->C64.ell, dg32};
  }

  // ---- hub rows (DIAG family, CSR): skewed degrees
  CK(build_hubs(p, d.hub_min_degree, true));

  // ---- edge adjacency (host build, one upload)
  if (d.cons_kind == ALM_BM_CONS_TRACE_EDGES) {
    const long E = d.n_edges;
    std::vector<int32_t> ei(E), ej(E);
    if (E) {
      HK(hipMemcpy(ei.data(), d.edge_i, E * sizeof(int32_t), hipMemcpyDeviceToHost));
      HK(hipMemcpy(ej.data(), d.edge_j, E * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    for (long e = 0; e < E; ++e) {
      if (ei[e] < 0 || ej[e] >= n || ei[e] >= ej[e])
        return bail(fail(ALM_BM_ERR_INVALID_PATTERN, "edge " + std::to_string(e) + ": need 0 <= i < j < n"));
      if (e > 0 && (ei[e] < ei[e - 1] || (ei[e] == ei[e - 1] && ej[e] <= ej[e - 1])))
        return bail(fail(ALM_BM_ERR_INVALID_PATTERN, "edges must be sorted by (i, j) without duplicates"));
    }
    std::vector<int32_t> urp(n + 1, 0), rp(n + 1, 0), ci(2 * E), eid(2 * E);
    for (long e = 0; e < E; ++e) {
      urp[ei[e] + 1]++;
      rp[ei[e] + 1]++;
      rp[ej[e] + 1]++;
    }
    for (long i = 0; i < n; ++i) {
      urp[i + 1] += urp[i];
      rp[i + 1] += rp[i];
    }
    std::vector<int32_t> cur(rp.begin(), rp.end() - 1);
    for (long e = 0; e < E; ++e) {  // lower entries: row j, column i < j
      ci[cur[ej[e]]] = ei[e];
      eid[cur[ej[e]]++] = (int32_t)e;
    }
    for (long e = 0; e < E; ++e) {  // upper entries: row i, column j > i
      ci[cur[ei[e]]] = ej[e];
      eid[cur[ei[e]]++] = (int32_t)e;
    }
    int32_t *drp, *dci, *deid, *durp;
    CK(dalloc_t(p, &drp, n + 1));
    CK(dalloc_t(p, &durp, n + 1));
    CK(dalloc_t(p, &dci, std::max<long>(1, 2 * E)));
    CK(dalloc_t(p, &deid, std::max<long>(1, 2 * E)));
    HK(hipMemcpy(drp, rp.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    HK(hipMemcpy(durp, urp.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    if (E) {
      HK(hipMemcpy(dci, ci.data(), 2 * E * sizeof(int32_t), hipMemcpyHostToDevice));
      HK(hipMemcpy(deid, eid.data(), 2 * E * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    p->adj = EdgeAdj{drp, dci, deid, durp, d.edge_j, (float)(2.0 * (double)d.n_edges / (double)std::max<long>(1, d.n))};
    CK(dalloc_t(p, &p->wE, std::max<long>(1, E)));
    CK(dalloc_t(p, &p->part2, (size_t)64 * (NUM_P + kMaxR)));
  }

  // ---- workspace
  p->nblk = row_blocks(n);
  p->max_blocks = std::max(p->nblk, max_row_blocks(n));
  // long edge-family rows (each split over a whole wave) need more, shorter blocks to fill the chip
  if (d.cons_kind == ALM_BM_CONS_TRACE_EDGES && p->adj.avg_deg >= 32.f) p->nblk = max_row_blocks(n);
  const size_t es = esize(d.precision);
  CK(dalloc_t(p, &p->part, (size_t)p->max_blocks * (NUM_P + kMaxR)));
  CK(dalloc_t(p, &p->part_c2, (size_t)p->max_blocks));
  CK(dalloc_t(p, &p->sc_api, 1));
  CK(dalloc_t(p, &p->sc_solve, 1));
  CK(dalloc(p, &p->G, (size_t)n * d.r_max * es));
  CK(dalloc(p, &p->Rtmp, (size_t)n * d.r_max * es));
  CK(dalloc(p, &p->Qbuf, (size_t)n * d.r_max * (d.precision == ALM_BM_F64 ? 8 : 4)));
  CK(dalloc_t(p, &p->Av, d.m));
  CK(dalloc_t(p, &p->ybuf, d.m));
  p->lnb = vec_blocks(n);
  CK(dalloc_t(p, &p->part_vec, (size_t)std::max(p->lnb, dual_blocks(d.m)) * 2 + 16));
  {
    hipError_t e = hipHostMalloc((void**)&p->sc_host, sizeof(DevScalars), hipHostMallocDefault);
    if (e != hipSuccess) return bail(fail(ALM_BM_ERR_OOM, "hipHostMalloc failed"));
    std::memset(p->sc_host, 0, sizeof(DevScalars));
  }
  HK(hipMemcpy(p->sc_api, p->sc_host, sizeof(DevScalars), hipMemcpyHostToDevice));
  HK(hipMemcpy(p->sc_solve, p->sc_host, sizeof(DevScalars), hipMemcpyHostToDevice));
  p->kmax = d.lanczos_kmax;
  if (p->kmax > 0) {
    CK(dalloc_t(p, &p->Q, (size_t)n * (p->kmax + 1)));
    CK(dalloc_t(p, &p->lw, n));
    CK(dalloc_t(p, &p->lv, n));
    CK(dalloc_t(p, &p->lh1, p->kmax + 1));
    CK(dalloc_t(p, &p->lh2, p->kmax + 1));
    CK(dalloc_t(p, &p->lalpha, p->kmax + 1));
    CK(dalloc_t(p, &p->lbeta, p->kmax + 1));
    CK(dalloc_t(p, &p->ls, p->kmax + 1));
    CK(dalloc_t(p, &p->lscal, 8));
    CK(dalloc_t(p, &p->lpart, (size_t)p->lnb * (p->kmax + 1)));
    CK(dalloc_t(p, &p->lpart2, (size_t)p->lnb));
    CK(dalloc_t(p, &p->bk_h, (size_t)(p->kmax + 1) * (p->kmax + 1)));
    CK(dalloc_t(p, &p->bk_colsum, (size_t)(p->kmax + 1)));
    CK(dalloc_t(p, &p->bk_coef, (size_t)(p->kmax + 1) * kMaxBlockQ));
  }
  // ---- workspace of optional solve features, reserved here so that no later
  // call allocates: block rank step, L-BFGS rings, the BF16 ladder's float factor
  if (d.rank_block_max > 1 && p->kmax > 0) {
    const int q = d.rank_block_max;
    const int np = q * (q + 1) / 2, ne = np * (np + 1) / 2;
    CK(dalloc_t(p, &p->vblk, (size_t)n * q));
    CK(dalloc_t(p, &p->ycoef, (size_t)q * std::max(p->kmax + 1, q)));
    CK(dalloc_t(p, &p->gpart, (size_t)p->lnb * ne));
  }
  if (d.lbfgs_memory_max > 0) {
    // ring elements: double for FP64 handles, bfloat16 otherwise (RingT); a
    // batch replaces the single state by one per instance
    const size_t lbe = d.precision == ALM_BM_F64 ? sizeof(double) : sizeof(bf16);
    p->lb_stride = ((long)n * d.r_max + 63) / 64 * 64;
    const size_t bytes = (size_t)(d.lbfgs_memory_max + 1) * (size_t)p->lb_stride * lbe;
    CK(dalloc(p, &p->lb_e, bytes));
    CK(dalloc(p, &p->lb_y, bytes));
    CK(dalloc_t(p, &p->lbs, 1));
    HK(hipMemset(p->lb_e, 0, bytes));
    HK(hipMemset(p->lb_y, 0, bytes));
  }
  if (d.precision == ALM_BM_BF16) {
    const size_t bytes = (size_t)n * d.r_max * sizeof(float);
    CK(dalloc(p, &p->R32, bytes));
    CK(dalloc(p, &p->G32, bytes));
    CK(dalloc(p, &p->Rt32, bytes));
  }
  HK(hipStreamCreateWithFlags(&p->ss, hipStreamNonBlocking));
  HK(hipStreamSynchronize(st));
  HK(hipGetLastError());
  *out = p;
  return ALM_BM_OK;
#undef CK
#undef HK
}

extern "C" alm_bm_status alm_bm_destroy(alm_bm_problem* p) {
  if (!p) return ALM_BM_OK;
  (void)hipDeviceSynchronize();
  free_all(p);
  delete p;
  return ALM_BM_OK;
}

// --------------------------------------------------------------------- enqueue helpers

// f, G (nullable), Av (nullable) at (R, y): one objective/gradient evaluation.
template <typename T>
static void enqueue_objgrad(alm_bm_problem* p, int r, const T* R, const double* y, double sigma, T* G, double* Av,
                            DevScalars* sc, int mode, double* f_out, hipStream_t st) {
  const auto& d = p->d;
  if (d.cons_kind == ALM_BM_CONS_DIAG) {
    launch_objgrad_diag<T>(cost_of<T>(p), r, p->variant, R, y, d.b, sigma, G, Av, p->part, sc, 0, p->tab, p->nblk,
                           st);
    launch_fin_objgrad(p->part, p->nblk, sc, sigma, mode, f_out, st, p->tab, p->count);
  } else {
    launch_edges_p1<T>(p->adj, d.n, r, p->variant, R, y, d.b, sigma, Av, p->wE, p->part, sc, p->nblk, st, p->rho);
    launch_fin_edges1(p->part, p->nblk, r, sc, y, d.b, sigma, d.trace_coef, Av, st, p->part2);
    launch_edges_p2<T>(cost_of<T>(p), p->adj, r, p->variant, R, p->wE, d.trace_coef, d.j_coef, nullptr, G, p->part,
                       sc, p->nblk, st);
    launch_fin_edges2(p->part, p->nblk, r, sc, sigma, mode, f_out, st, p->part2);
  }
}

// One inner gradient step (flag-guarded, decisions taken on the device):
// DIAG family: apply the pending step and evaluate the new gradient from the
// carried cost product (or, every `refresh` steps, with the full sparse pass),
// stop test, line-search product Q = C G, step choice.  One sparse product per
// step except on refresh steps.
// TRACE_EDGES family: full evaluation, stop test, line search, update.
template <typename T>
static void enqueue_inner_step(alm_bm_problem* p, int r, T* R, const double* y, double sigma, T* G, int refresh,
                               hipStream_t st) {
  using V = typename Acc<T>::type;
  const auto& d = p->d;
  DevScalars* sc = p->sc_solve;
  if (d.cons_kind == ALM_BM_CONS_DIAG) {
    V* Q = static_cast<V*>(p->Qbuf);
    using S = RingT<T>;
    const LbfgsRing<S> lb = lbfgs_ring<S>(p);  // empty: gradient descent
    launch_upd_eval_diag<T>(d.n, r, p->variant, R, G, Q, y, d.b, sigma, p->Av, p->part, sc, refresh, p->tab, p->nblk,
                            st, lb);
    launch_objgrad_diag<T>(cost_of<T>(p), r, p->variant, R, y, d.b, sigma, G, p->Av, p->part, sc, refresh, p->tab,
                           p->nblk, st, lb);
    launch_fin_objgrad(p->part, p->nblk, sc, sigma, 1, nullptr, st, p->tab, p->count);
    if (lb.s) {
      // L-BFGS: the direction E = H G and its line-search totals replace G's;
      // the line-search product gathers E in the ring type
      launch_lbfgs_dots<T>((long)d.n * r, r, G, lb, p->part, p->nblk, sc, st);
      launch_fin_lbfgs(p->part, p->nblk, sc, lb.s, st);
      launch_lbfgs_combine<T>(d.n, r, p->variant, R, G, y, d.b, sigma, p->Av, lb, p->part, sc, p->nblk, st);
      launch_fin_lsdir(p->part, p->nblk, sc, lb.s, st);
      launch_quadq_diag<S>(cost_of<S>(p), r, p->variant, lb.e, Q, p->part_c2, sc, p->tab, p->nblk, st, lb);
    } else {
      launch_quadq_diag<T>(cost_of<T>(p), r, p->variant, G, Q, p->part_c2, sc, p->tab, p->nblk, st);
    }
    launch_fin_step(p->part_c2, p->nblk, 1, sc, sigma, 0.0, 1, nullptr, nullptr, st, p->tab, p->count);
  } else {
    enqueue_objgrad<T>(p, r, R, y, sigma, G, p->Av, sc, 1, nullptr, st);
    launch_edges_p3<T>(cost_of<T>(p), p->adj, r, p->variant, R, G, y, d.b, p->Av, p->part, sc, p->nblk, st,
                       p->rho);
    launch_fin_edges3(p->part, p->nblk, r, sc, y, d.b, sigma, d.trace_coef, d.j_coef, 1, nullptr, nullptr, st,
                      p->part2);
    launch_update<T>((long)d.n * r, R, G, sc, 1, st);
  }
}

static int default_refresh(alm_bm_precision prec) {
  return prec == ALM_BM_F64 ? 32 : (prec == ALM_BM_F32 ? 16 : 8);
}

// Subproblem solver of a solve: checks the options against the handle's
// workspace; the returned memory is 0 for gradient descent.
static alm_bm_status check_inner(const alm_bm_problem* p, const alm_bm_options& o, int& lb_m) {
  lb_m = 0;
  if (o.inner_solver == ALM_BM_INNER_GD) return ALM_BM_OK;
  if (o.inner_solver != ALM_BM_INNER_LBFGS) return fail(ALM_BM_ERR_INVALID_ARG, "unknown inner_solver");
  if (p->d.cons_kind != ALM_BM_CONS_DIAG || p->tab.inst)
    return fail(ALM_BM_ERR_UNSUPPORTED, "the L-BFGS inner solver is for single DIAG-family problems");
  if (o.lbfgs_memory < 1 || o.lbfgs_memory > p->d.lbfgs_memory_max)
    return fail(ALM_BM_ERR_INVALID_ARG, "lbfgs_memory must be in 1..lbfgs_memory_max of the handle (" +
                                            std::to_string(p->d.lbfgs_memory_max) + ")");
  lb_m = o.lbfgs_memory;
  return ALM_BM_OK;
}

// Sets the handle's L-BFGS memory for the length of one solve.
struct InnerScope {
  alm_bm_problem* p;
  InnerScope(alm_bm_problem* p_, int m) : p(p_) { p->lb_m = m; }
  ~InnerScope() { p->lb_m = 0; }
};

static alm_bm_status check_r(const alm_bm_problem* p, int r) {
  if (r < 1 || r > p->d.r_max) return fail(ALM_BM_ERR_INVALID_ARG, "r must be in 1..r_max");
  return ALM_BM_OK;
}

// --------------------------------------------------------------------- API: per call

extern "C" alm_bm_status alm_bm_objective_grad(alm_bm_problem* p, int32_t r, const void* R, const double* y,
                                               double sigma, double* f, void* G, double* Av, hipStream_t st) {
  if (!p || !R || !y || !f) return fail(ALM_BM_ERR_INVALID_ARG, "objective_grad: null argument");
  STCHK(check_r(p, r));
  with_storage(p->d.precision, [&]<typename T>() {
    enqueue_objgrad<T>(p, r, static_cast<const T*>(R), y, sigma, static_cast<T*>(G), Av, p->sc_api, 0, f, st);
    return 0;
  });
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_cost_apply(alm_bm_problem* p, int32_t r, const void* X, void* P, double* xpx,
                                           hipStream_t st) {
  if (!p || !X || !P) return fail(ALM_BM_ERR_INVALID_ARG, "cost_apply: null argument");
  STCHK(check_r(p, r));
  if (p->d.j_coef != 0.0) return fail(ALM_BM_ERR_UNSUPPORTED, "cost_apply: cost with a -J term");
  with_storage(p->d.precision, [&]<typename T>() {
    using V = typename Acc<T>::type;
    launch_quadq_diag<T>(cost_of<T>(p), r, p->variant, static_cast<const T*>(X), static_cast<V*>(P), p->part_c2,
                         nullptr, p->tab, p->nblk, st);
    if (xpx) launch_fin_sum(p->part_c2, p->nblk, xpx, 0, st);
    return 0;
  });
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_line_search(alm_bm_problem* p, int32_t r, const void* R, const void* G,
                                            const double* y, double sigma, double* coeffs, double* t_star,
                                            hipStream_t st) {
  if (!p || !R || !G || !y || !coeffs) return fail(ALM_BM_ERR_INVALID_ARG, "line_search: null argument");
  STCHK(check_r(p, r));
  const auto& d = p->d;
  with_storage(d.precision, [&]<typename T>() {
    const T* Rt = static_cast<const T*>(R);
    const T* Gt = static_cast<const T*>(G);
    if (d.cons_kind == ALM_BM_CONS_DIAG) {
      launch_ls_diag<T>(cost_of<T>(p), r, p->variant, Rt, Gt, y, d.b, p->part, p->nblk, st);
      launch_fin_ls(p->part, p->nblk, p->sc_api, sigma, coeffs, t_star, st);
    } else {
      DevScalars* sc = p->sc_api;
      launch_edges_p1<T>(p->adj, d.n, r, p->variant, Rt, y, d.b, sigma, p->Av, p->wE, p->part, sc, p->nblk, st);
      launch_fin_edges1(p->part, p->nblk, r, sc, y, d.b, sigma, d.trace_coef, p->Av, st, p->part2);
      launch_edges_p2<T>(cost_of<T>(p), p->adj, r, p->variant, Rt, p->wE, d.trace_coef, d.j_coef, Gt, nullptr,
                         p->part, sc, p->nblk, st);
      launch_fin_edges2(p->part, p->nblk, r, sc, sigma, 0, nullptr, st, p->part2);
      launch_edges_p3<T>(cost_of<T>(p), p->adj, r, p->variant, Rt, Gt, y, d.b, p->Av, p->part, sc, p->nblk, st);
      launch_fin_edges3(p->part, p->nblk, r, sc, y, d.b, sigma, d.trace_coef, d.j_coef, 0, coeffs, t_star, st,
                        p->part2);
    }
    return 0;
  });
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_gd_step(alm_bm_problem* p, int32_t r, void* R, const double* y, double sigma,
                                        double* f, double* t, void* G, hipStream_t st) {
  if (!p || !R || !y) return fail(ALM_BM_ERR_INVALID_ARG, "gd_step: null argument");
  STCHK(check_r(p, r));
  const auto& d = p->d;
  with_storage(d.precision, [&]<typename T>() {
    T* Rt = static_cast<T*>(R);
    T* Gt = G ? static_cast<T*>(G) : static_cast<T*>(p->G);
    DevScalars* sc = p->sc_api;
    enqueue_objgrad<T>(p, r, Rt, y, sigma, Gt, p->Av, sc, 0, f, st);
    if (d.cons_kind == ALM_BM_CONS_DIAG) {
      launch_quad_diag<T>(cost_of<T>(p), r, p->variant, Gt, p->part_c2, sc, p->nblk, st);
      launch_fin_step(p->part_c2, p->nblk, 1, sc, sigma, 0.0, 0, nullptr, t, st);
    } else {
      launch_edges_p3<T>(cost_of<T>(p), p->adj, r, p->variant, Rt, Gt, y, d.b, p->Av, p->part, sc, p->nblk, st);
      launch_fin_edges3(p->part, p->nblk, r, sc, y, d.b, sigma, d.trace_coef, d.j_coef, 0, nullptr, t, st, p->part2);
    }
    launch_update<T>((long)d.n * r, Rt, Gt, sc, 0, st);
    return 0;
  });
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_dual_update(alm_bm_problem* p, const double* Av, double sigma, double* y,
                                            double* pinf, hipStream_t st) {
  if (!p || !Av || !y) return fail(ALM_BM_ERR_INVALID_ARG, "dual_update: null argument");
  launch_dual(p->d.m, Av, p->d.b, y, y, sigma, p->part_vec, p->sc_api, p->bnorm, pinf, st);
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

// --------------------------------------------------------------------- warm start

extern "C" alm_bm_status alm_bm_ws_features(alm_bm_problem* p, float* feats, float* scratch, hipStream_t st) {
  if (!p || !feats || !scratch) return fail(ALM_BM_ERR_INVALID_ARG, "ws_features: null argument");
  if (p->d.cons_kind != ALM_BM_CONS_DIAG) return fail(ALM_BM_ERR_UNSUPPORTED, "ws_features: DIAG family only");
  launch_ws_features(p->C64, feats, scratch, st);
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_ws_pool(const float* feats, int64_t n, double* out, double* work, hipStream_t st) {
  if (!feats || !out || !work || n < 1) return fail(ALM_BM_ERR_INVALID_ARG, "ws_pool: bad argument");
  launch_ws_pool(feats, n, work, 64, out, st);  // 64 blocks x 8 partials
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" int64_t alm_bm_ws_param_count(int32_t n_in, int32_t h) { return ws_param_count(n_in, h); }

extern "C" int64_t alm_bm_ws_work_size(int32_t n_in, int32_t h, int32_t nblocks) {
  // per-block gradient partials, then per-block losses as doubles (2 floats each)
  return (int64_t)nblocks * ws_param_count(n_in, h) + 2 * (int64_t)nblocks + 2;
}

static bool ws_shape_ok(int32_t n_in, int32_t h) {
  return n_in >= 1 && n_in <= ALM_BM_WS_NFEAT && (h == 16 || h == 32 || h == 64);
}

extern "C" alm_bm_status alm_bm_ws_forward(const float* params, int32_t n_in, int32_t h, const float* mu,
                                           const float* inv_sd, int64_t n, const float* X, double* out,
                                           hipStream_t st) {
  if (!params || !mu || !inv_sd || !X || !out || n < 0) return fail(ALM_BM_ERR_INVALID_ARG, "ws_forward: bad argument");
  if (!ws_shape_ok(n_in, h)) return fail(ALM_BM_ERR_INVALID_ARG, "ws_forward: n_in <= 8 and h in {16,32,64}");
  if (n == 0) return ALM_BM_OK;
  launch_ws_forward(params, n_in, h, mu, inv_sd, n, X, out, st);
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_ws_loss_grad(const float* params, int32_t n_in, int32_t h, const float* mu,
                                             const float* inv_sd, int64_t n, const float* X, const float* target,
                                             float* grad, double* loss, float* work, int32_t nblocks,
                                             hipStream_t st) {
  if (!params || !mu || !inv_sd || !X || !target || !grad || !work || n < 1)
    return fail(ALM_BM_ERR_INVALID_ARG, "ws_loss_grad: bad argument");
  if (!ws_shape_ok(n_in, h)) return fail(ALM_BM_ERR_INVALID_ARG, "ws_loss_grad: n_in <= 8 and h in {16,32,64}");
  if (nblocks < 1 || nblocks > 4096) return fail(ALM_BM_ERR_INVALID_ARG, "ws_loss_grad: nblocks in 1..4096");
  const int np = ws_param_count(n_in, h);
  float* gpart = work;
  // doubles after the float partials, 8-byte aligned
  size_t off = (size_t)nblocks * np;
  off = (off + 1) & ~(size_t)1;
  double* lpart = reinterpret_cast<double*>(work + off);
  launch_ws_backward(params, n_in, h, mu, inv_sd, n, X, target, gpart, lpart, nblocks, grad, loss, st);
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_ws_adam(float* params, const float* grad, float* m, float* v, int32_t count, float lr,
                                        float beta1, float beta2, float eps, int32_t step, hipStream_t st) {
  if (!params || !grad || !m || !v || count < 1 || step < 1) return fail(ALM_BM_ERR_INVALID_ARG, "ws_adam: bad argument");
  launch_ws_adam(params, grad, m, v, count, lr, beta1, beta2, eps, step, st);
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_ws_ridge_fit(const double* X, const double* t, int32_t k, int32_t p, double lambda,
                                             double* coef) {
  if (!X || !t || !coef || k < 1 || p < 0 || p > 64 || lambda < 0.0)
    return fail(ALM_BM_ERR_INVALID_ARG, "ws_ridge_fit: bad argument");
  const int q = p + 1;  // with intercept (not penalised)
  std::vector<double> A(q * q, 0.0), rhs(q, 0.0);
  for (int r = 0; r < k; ++r) {
    for (int i = 0; i < q; ++i) {
      const double xi = i < p ? X[(long)r * p + i] : 1.0;
      rhs[i] += xi * t[r];
      for (int j = 0; j < q; ++j) A[i * q + j] += xi * (j < p ? X[(long)r * p + j] : 1.0);
    }
  }
  for (int i = 0; i < p; ++i) A[i * q + i] += lambda;
  // Gaussian elimination with partial pivoting
  for (int c = 0; c < q; ++c) {
    int piv = c;
    for (int r = c + 1; r < q; ++r)
      if (std::fabs(A[r * q + c]) > std::fabs(A[piv * q + c])) piv = r;
    if (std::fabs(A[piv * q + c]) < 1e-300) return fail(ALM_BM_ERR_NUMERIC, "ws_ridge_fit: singular system");
    if (piv != c) {
      for (int j = 0; j < q; ++j) std::swap(A[c * q + j], A[piv * q + j]);
      std::swap(rhs[c], rhs[piv]);
    }
    for (int r = c + 1; r < q; ++r) {
      const double f = A[r * q + c] / A[c * q + c];
      for (int j = c; j < q; ++j) A[r * q + j] -= f * A[c * q + j];
      rhs[r] -= f * rhs[c];
    }
  }
  for (int c = q - 1; c >= 0; --c) {
    double s = rhs[c];
    for (int j = c + 1; j < q; ++j) s -= A[c * q + j] * coef[j];
    coef[c] = s / A[c * q + c];
  }
  return ALM_BM_OK;
}

// --------------------------------------------------------------------- tiling

extern "C" alm_bm_status alm_bm_set_tiles(alm_bm_problem* p, int32_t variant, int32_t row_blocks_) {
  if (!p) return fail(ALM_BM_ERR_INVALID_ARG, "set_tiles: null handle");
  if (variant < 0 || variant > 2) return fail(ALM_BM_ERR_INVALID_ARG, "set_tiles: variant must be 0..2");
  int nb = row_blocks_ == 0 ? row_blocks(p->d.n) : row_blocks_;
  if (nb < 8 || nb % 8 != 0 || nb > p->max_blocks)
    return fail(ALM_BM_ERR_INVALID_ARG, "set_tiles: row_blocks must be a multiple of 8 in [8, " +
                                            std::to_string(p->max_blocks) + "]");
  p->variant = variant;
  p->nblk = nb;
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_set_hub_threshold(alm_bm_problem* p, int32_t min_degree, int32_t* hubs_out) {
  if (!p) return fail(ALM_BM_ERR_INVALID_ARG, "set_hub_threshold: null handle");
  if (p->tab.inst) return fail(ALM_BM_ERR_UNSUPPORTED, "set_hub_threshold: not on a batch");
  STCHK(build_hubs(p, min_degree, false));
  if (hubs_out) *hubs_out = p->C64.nh;
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_autotune(alm_bm_problem* p, int32_t r, int32_t reps, int32_t* variant_out,
                                         int32_t* blocks_out, hipStream_t st) {
  if (!p) return fail(ALM_BM_ERR_INVALID_ARG, "autotune: null handle");
  STCHK(check_r(p, r));
  if (reps < 1) return fail(ALM_BM_ERR_INVALID_ARG, "autotune: reps < 1");
  const auto& d = p->d;
  HIPCHK(hipMemsetAsync(p->Rtmp, 0, (size_t)d.n * r * esize(d.precision), st));
  HIPCHK(hipMemsetAsync(p->ybuf, 0, (size_t)d.m * sizeof(double), st));
  std::vector<int> cands;
  for (int nb : {row_blocks(d.n), 1024, 2048, 4096, 8192, 16384})
    if (nb >= 8 && nb % 8 == 0 && nb <= p->max_blocks &&
        std::find(cands.begin(), cands.end(), nb) == cands.end())
      cands.push_back(nb);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best = INFINITY;
  int bv = p->variant, bb = p->nblk;
  for (int v = 0; v <= 2; ++v) {
    for (int nb : cands) {
      p->variant = v;
      p->nblk = nb;
      auto run = [&]() {
        with_storage(d.precision, [&]<typename T>() {
          enqueue_objgrad<T>(p, r, static_cast<const T*>(p->Rtmp), p->ybuf, 1.0, static_cast<T*>(p->G), p->Av,
                             p->sc_api, 0, nullptr, st);
          return 0;
        });
      };
      run();  // warm
      HIPCHK(hipEventRecord(e0, st));
      for (int k = 0; k < reps; ++k) run();
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        bv = v;
        bb = nb;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->variant = bv;
  p->nblk = bb;
  if (variant_out) *variant_out = bv;
  if (blocks_out) *blocks_out = bb;
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

// --------------------------------------------------------------------- Lanczos

static int sturm_count(const std::vector<double>& a, const std::vector<double>& b, int m, double x) {
  double bmax = 0.0;
  for (int i = 0; i + 1 < m; ++i) bmax = std::max(bmax, b[i] * b[i]);
  const double pivmin = DBL_MIN * std::max(1.0, bmax);
  int c = 0;
  double q = a[0] - x;
  if (std::fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++c;
  for (int i = 1; i < m; ++i) {
    q = a[i] - x - b[i - 1] * b[i - 1] / q;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++c;
  }
  return c;
}

// Smallest eigenvalue of the symmetric tridiagonal (a[0..m), b[0..m-1)) by
// Sturm-sequence bisection.
static double tri_min_eig(const std::vector<double>& a, const std::vector<double>& b, int m) {
  if (m == 1) return a[0];
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < m; ++i) {
    const double rad = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - rad);
    hi = std::max(hi, a[i] + rad);
  }
  const double scale = std::max(std::fabs(lo), std::fabs(hi));
  for (int it = 0; it < 300; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (hi - lo <= 2.0 * DBL_EPSILON * scale || mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, m, mid) >= 1) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Eigenvector of the tridiagonal for eigenvalue theta by inverse iteration,
// (T - theta I) factored by Gaussian elimination with partial pivoting.
static void tri_eigvec(const std::vector<double>& a, const std::vector<double>& b, int m, double theta,
                       std::vector<double>& z) {
  z.assign(m, 0.0);
  if (m == 1) {
    z[0] = 1.0;
    return;
  }
  double tnorm = 0.0;
  for (int i = 0; i < m; ++i) tnorm = std::max(tnorm, std::fabs(a[i]) + (i + 1 < m ? std::fabs(b[i]) : 0.0));
  const double tiny = std::max(tnorm, 1e-300) * DBL_EPSILON;
  std::vector<double> dl(m - 1), dd(m), du(m - 1), du2(std::max(1, m - 2), 0.0);
  std::vector<char> swp(m - 1, 0);
  for (int i = 0; i < m; ++i) dd[i] = a[i] - theta;
  for (int i = 0; i + 1 < m; ++i) dl[i] = du[i] = b[i];
  for (int i = 0; i + 1 < m; ++i) {
    if (std::fabs(dd[i]) >= std::fabs(dl[i])) {
      if (dd[i] == 0.0) dd[i] = tiny;
      const double fact = dl[i] / dd[i];
      dl[i] = fact;
      dd[i + 1] -= fact * du[i];
      if (i + 2 < m) du2[i] = 0.0;
    } else {
      const double fact = dd[i] / dl[i];
      dd[i] = dl[i];
      dl[i] = fact;
      const double temp = du[i];
      du[i] = dd[i + 1];
      dd[i + 1] = temp - fact * dd[i + 1];
      if (i + 2 < m) {
        du2[i] = du[i + 1];
        du[i + 1] = -fact * du[i + 1];
      }
      swp[i] = 1;
    }
  }
  if (dd[m - 1] == 0.0) dd[m - 1] = tiny;
  for (int i = 0; i < m; ++i) z[i] = 1.0 + 0.01 * (double)((i * 7919) % 97) / 97.0;
  for (int it = 0; it < 4; ++it) {
    std::vector<double> x = z;
    for (int i = 0; i + 1 < m; ++i) {
      if (swp[i]) {
        const double t = x[i];
        x[i] = x[i + 1];
        x[i + 1] = t - dl[i] * x[i];
      } else {
        x[i + 1] -= dl[i] * x[i];
      }
    }
    x[m - 1] /= dd[m - 1];
    x[m - 2] = (x[m - 2] - du[m - 2] * x[m - 1]) / dd[m - 2];
    for (int i = m - 3; i >= 0; --i) x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / dd[i];
    double nrm = 0.0;
    for (double v : x) nrm += v * v;
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) break;
    for (int i = 0; i < m; ++i) z[i] = x[i] / nrm;
  }
}

// Eigen-decomposition of a small symmetric q x q matrix (row-major) by cyclic
// Jacobi rotations: A = U diag(lam) U^T, U row-major with eigenvectors in columns.
static void small_sym_eig(int q, std::vector<double> A, std::vector<double>& lam, std::vector<double>& U) {
  U.assign(q * q, 0.0);
  for (int i = 0; i < q; ++i) U[i * q + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        tot += A[i * q + j] * A[i * q + j];
        if (i != j) off += A[i * q + j] * A[i * q + j];
      }
    if (off <= 1e-30 * std::max(tot, 1e-300)) break;
    for (int p0 = 0; p0 < q; ++p0)
      for (int q0 = p0 + 1; q0 < q; ++q0) {
        const double apq = A[p0 * q + q0];
        if (apq == 0.0) continue;
        const double tau = (A[q0 * q + q0] - A[p0 * q + p0]) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < q; ++k) {  // A <- A J (columns p0, q0)
          const double akp = A[k * q + p0], akq = A[k * q + q0];
          A[k * q + p0] = c * akp - s * akq;
          A[k * q + q0] = s * akp + c * akq;
        }
        for (int k = 0; k < q; ++k) {  // A <- J^T A (rows p0, q0)
          const double apk = A[p0 * q + k], aqk = A[q0 * q + k];
          A[p0 * q + k] = c * apk - s * aqk;
          A[q0 * q + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < q; ++k) {
          const double ukp = U[k * q + p0], ukq = U[k * q + q0];
          U[k * q + p0] = c * ukp - s * ukq;
          U[k * q + q0] = s * ukp + c * ukq;
        }
      }
  }
  lam.resize(q);
  for (int i = 0; i < q; ++i) lam[i] = A[i * q + i];
}

// Nearest PSD matrix (eigenvalues clipped at zero).
static std::vector<double> psd_clip(int q, const std::vector<double>& M) {
  std::vector<double> sym(q * q), lam, U, out(q * q, 0.0);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) sym[i * q + j] = 0.5 * (M[i * q + j] + M[j * q + i]);
  small_sym_eig(q, sym, lam, U);
  for (int k = 0; k < q; ++k) {
    if (!(lam[k] > 0.0)) continue;
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) out[i * q + j] += lam[k] * U[i * q + k] * U[j * q + k];
  }
  return out;
}

// The block rank step's subproblem (Alg. 1): minimise over S PSD (q x q)
//   phi(S) = sum_a theta_a S_aa + sigma/2 sum_{abcd} S_ab S_cd M4[ab, cd],
// M4[ab, cd] = sum_i V_ia V_ib V_ic V_id (symmetric in every index), which is
// <Z V, V> S plus the penalty of A(V S V^T) for Ritz directions V of Z (then
// V^T Z V = diag(theta)).  Accelerated projected gradient with monotone
// restarts, step 1 / L (L from power iteration on the Hessian map).
static std::vector<double> block_subproblem(int q, const std::vector<double>& theta,
                                            const std::vector<double>& M4, int np, double sigma) {
  std::vector<int> pid(q * q);
  for (int a = 0, k = 0; a < q; ++a)
    for (int b = a; b < q; ++b, ++k) pid[a * q + b] = pid[b * q + a] = k;
  auto hess = [&](const std::vector<double>& S) {  // S -> sigma M4 . S (Frobenius gradient of the quadratic)
    std::vector<double> out(q * q, 0.0);
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b) {
        double s = 0.0;
        for (int c = 0; c < q; ++c)
          for (int d = 0; d < q; ++d) s += M4[(size_t)pid[a * q + b] * np + pid[c * q + d]] * S[c * q + d];
        out[a * q + b] = sigma * s;
      }
    return out;
  };
  auto dot = [&](const std::vector<double>& X, const std::vector<double>& Y) {
    double s = 0.0;
    for (int i = 0; i < q * q; ++i) s += X[i] * Y[i];
    return s;
  };
  auto phi = [&](const std::vector<double>& S) {
    double lin = 0.0;
    for (int a = 0; a < q; ++a) lin += theta[a] * S[a * q + a];
    return lin + 0.5 * dot(S, hess(S));
  };
  auto grad = [&](const std::vector<double>& S) {
    std::vector<double> g = hess(S);
    for (int a = 0; a < q; ++a) g[a * q + a] += theta[a];
    return g;
  };
  // largest eigenvalue of the Hessian map on symmetric matrices
  std::vector<double> X(q * q, 0.0);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) X[i * q + j] = (i == j ? 1.0 : 0.1) / q;
  double L = 0.0;
  for (int it = 0; it < 300; ++it) {
    std::vector<double> Y = hess(X);
    const double nrm = std::sqrt(dot(Y, Y));
    if (!(nrm > 0.0)) break;
    L = dot(X, Y) / dot(X, X);
    for (int i = 0; i < q * q; ++i) X[i] = Y[i] / nrm;
  }
  std::vector<double> S(q * q, 0.0);
  if (!(L > 0.0)) return S;
  L *= 1.05;
  std::vector<double> Yk = S;
  double t = 1.0, fS = phi(S);
  for (int it = 0; it < 20000; ++it) {
    std::vector<double> g = grad(Yk), Sn(q * q);
    for (int i = 0; i < q * q; ++i) Sn[i] = Yk[i] - g[i] / L;
    Sn = psd_clip(q, Sn);
    double fn = phi(Sn);
    if (fn > fS) {  // restart from S with a plain projected step
      g = grad(S);
      for (int i = 0; i < q * q; ++i) Sn[i] = S[i] - g[i] / L;
      Sn = psd_clip(q, Sn);
      fn = phi(Sn);
      t = 1.0;
    }
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    for (int i = 0; i < q * q; ++i) Yk[i] = Sn[i] + ((t - 1.0) / tn) * (Sn[i] - S[i]);
    double ds = 0.0, ns = 0.0;
    for (int i = 0; i < q * q; ++i) {
      ds += (Sn[i] - S[i]) * (Sn[i] - S[i]);
      ns += Sn[i] * Sn[i];
    }
    S = Sn;
    fS = fn;
    t = tn;
    if (std::sqrt(ds) <= 1e-13 * (1.0 + std::sqrt(ns)) && it > 10) break;
  }
  return S;
}

extern "C" alm_bm_status alm_bm_psd_step(int32_t q, const double* theta, const double* M4, double sigma,
                                         double* S) {
  if (q < 1 || q > 8 || !theta || !M4 || !S) return fail(ALM_BM_ERR_INVALID_ARG, "psd_step: bad arguments");
  if (!(sigma > 0.0)) return fail(ALM_BM_ERR_INVALID_ARG, "psd_step: sigma must be positive");
  const int np = q * (q + 1) / 2;
  const std::vector<double> th(theta, theta + q), m4(M4, M4 + (size_t)np * np);
  for (double v : m4)
    if (!std::isfinite(v)) return fail(ALM_BM_ERR_NUMERIC, "psd_step: non-finite M4");
  for (double v : th)
    if (!std::isfinite(v)) return fail(ALM_BM_ERR_NUMERIC, "psd_step: non-finite theta");
  const std::vector<double> out = block_subproblem(q, th, m4, np, sigma);
  std::copy(out.begin(), out.end(), S);
  return ALM_BM_OK;
}

struct LanczosOut {
  double theta = 0.0;
  double resid = 0.0;
  int iters = 0;
};

// Lanczos on Z(y) with two classical Gram-Schmidt passes per step; the Ritz
// vector for the smallest Ritz value goes to v (device, n).
static alm_bm_status lanczos_pass(alm_bm_problem* p, const double* y, int kmax, double tol, uint64_t seed,
                                  bool restart, double* v, LanczosOut& out, hipStream_t st) {
  const auto& d = p->d;
  const long n = d.n;
  const long ldq = n;
  const int nb = p->lnb;
  const int pstride = p->kmax + 1;
  kmax = std::min(kmax, p->kmax);
  if (kmax < 1) return fail(ALM_BM_ERR_INVALID_ARG, "lanczos: no Lanczos workspace (lanczos_kmax = 0)");
  kmax = (int)std::min<long>(kmax, n);
  double* qsum = (d.j_coef != 0.0) ? &p->sc_api->qsum : nullptr;
  const int cons = d.cons_kind == ALM_BM_CONS_DIAG ? 0 : 1;
  if (restart) {
    // restart from the previous (unit) Ritz vector in v
    launch_resid(n, v, v, 0.0, nullptr, p->lpart2, nb, st);
    launch_fin_sum(p->lpart2, nb, p->lscal, 1, st);
    launch_scale(n, v, p->lscal, p->Q, p->lpart2, nb, qsum, st);
  } else {
    launch_rand(n, seed, p->lw, p->lpart2, nb, st);
    launch_fin_sum(p->lpart2, nb, p->lscal, 1, st);
    launch_scale(n, p->lw, p->lscal, p->Q, p->lpart2, nb, qsum, st);
  }
  std::vector<double> ha(kmax + 1), hb(kmax + 1), z;
  int m = 0;
  double theta = 0.0;
  const int check_every = n <= 4096 ? 4 : 8;
  for (int j = 0; j < kmax; ++j) {
    const double* qj = p->Q + (long)j * ldq;
    launch_slack_mv(p->C64, cons, p->adj, y, d.trace_coef, d.j_coef, p->sc_api, qj, p->lw, st);
    launch_dots(n, j + 1, p->Q, ldq, p->lw, p->lpart, pstride, nb, p->lh1, st);
    launch_sub(n, j + 1, p->Q, ldq, p->lh1, p->lw, p->lpart2, nb, st);
    launch_dots(n, j + 1, p->Q, ldq, p->lw, p->lpart, pstride, nb, p->lh2, st);
    launch_sub(n, j + 1, p->Q, ldq, p->lh2, p->lw, p->lpart2, nb, st);
    launch_fin_ab(p->lpart2, nb, p->lh1, p->lh2, j, p->lalpha, p->lbeta, st);
    launch_scale(n, p->lw, p->lbeta + j, p->Q + (long)(j + 1) * ldq, p->lpart2, nb, qsum, st);
    const bool last = (j + 1 == kmax);
    if (((j + 1) % check_every) == 0 || last) {
      HIPCHK(hipMemcpyAsync(ha.data(), p->lalpha, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hb.data(), p->lbeta, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      double anorm = 0.0;
      for (int i = 0; i <= j; ++i) anorm = std::max(anorm, std::fabs(ha[i]) + std::fabs(hb[i]));
      for (int i = 0; i <= j; ++i)
        if (!std::isfinite(ha[i]) || !std::isfinite(hb[i])) return fail(ALM_BM_ERR_NUMERIC, "lanczos: NaN/Inf");
      // an (almost) invariant subspace ends the recurrence
      int mm = j + 1;
      bool breakdown = false;
      for (int i = 0; i <= j; ++i)
        if (hb[i] <= 1e-13 * std::max(anorm, 1e-300)) {
          mm = i + 1;
          breakdown = true;
          break;
        }
      theta = tri_min_eig(ha, hb, mm);
      tri_eigvec(ha, hb, mm, theta, z);
      m = mm;
      const double est = breakdown ? 0.0 : std::fabs(hb[mm - 1] * z[mm - 1]);
      if (breakdown || est <= tol || last) break;
    }
  }
  HIPCHK(hipMemcpyAsync(p->ls, z.data(), m * sizeof(double), hipMemcpyHostToDevice, st));
  launch_combine(n, m, p->Q, ldq, p->ls, v, p->lpart2, nb, st);
  launch_fin_sum(p->lpart2, nb, p->lscal + 1, 1, st);
  launch_scale(n, v, p->lscal + 1, v, p->lpart2, nb, qsum, st);
  launch_slack_mv(p->C64, cons, p->adj, y, d.trace_coef, d.j_coef, p->sc_api, v, p->lw, st);
  launch_resid(n, p->lw, v, theta, nullptr, p->lpart2, nb, st);
  launch_fin_sum(p->lpart2, nb, p->lscal + 2, 1, st);
  double hres = 0.0;
  HIPCHK(hipMemcpyAsync(&hres, p->lscal + 2, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  out.theta = theta;
  out.resid = hres;
  out.iters = m;
  if (!std::isfinite(theta)) return fail(ALM_BM_ERR_NUMERIC, "lanczos: non-finite Ritz value");
  return ALM_BM_OK;
}

// Lanczos with explicit restarts from the Ritz vector while its residual
// exceeds tol (a pass that stops at kmax without converging overestimates
// lambda_min; the restarts keep the KKT test and the rank test honest).
static alm_bm_status lanczos_run(alm_bm_problem* p, const double* y, int kmax, double tol, uint64_t seed, double* v,
                                 LanczosOut& out, hipStream_t st, int restarts = 3) {
  int total = 0;
  for (int rs = 0; rs <= restarts; ++rs) {
    STCHK(lanczos_pass(p, y, kmax, tol, seed, rs > 0, v, out, st));
    total += out.iters;
    if (out.resid <= tol) break;
  }
  out.iters = total;
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_lanczos_min_eig(alm_bm_problem* p, const double* y, int32_t max_iter, double tol,
                                                uint64_t seed, double* theta, double* v, double* resid,
                                                int32_t* iters, hipStream_t st) {
  if (!p || !y || !theta) return fail(ALM_BM_ERR_INVALID_ARG, "lanczos_min_eig: null argument");
  if (max_iter < 1) return fail(ALM_BM_ERR_INVALID_ARG, "lanczos_min_eig: max_iter < 1");
  if (max_iter > p->kmax) return fail(ALM_BM_ERR_INVALID_ARG, "lanczos_min_eig: max_iter > lanczos_kmax");
  LanczosOut o;
  STCHK(lanczos_run(p, y, max_iter, tol, seed, v ? v : p->lv, o, st));
  HIPCHK(hipMemcpyAsync(theta, &o.theta, sizeof(double), hipMemcpyHostToDevice, st));
  if (resid) HIPCHK(hipMemcpyAsync(resid, &o.resid, sizeof(double), hipMemcpyHostToDevice, st));
  if (iters) HIPCHK(hipMemcpyAsync(iters, &o.iters, sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return ALM_BM_OK;
}

// --------------------------------------------------------------------- block Krylov

// The q smallest Ritz pairs of Z(y) from the block Krylov space
// span{V0, Z V0, Z^2 V0, ...} (V0: q counter-based random vectors), m <=
// kmax + 1 orthonormal columns.  The columns are built one at a time: column c
// is Z q_{c-q} orthogonalised against columns 0..c-1 (two classical
// Gram-Schmidt passes) and normalised, which is the block Lanczos recurrence
// with full reorthogonalisation.  The first-pass coefficients are the entries
// q_i^T Z q_j (i <= j) of H = Q^T Z Q; the last q columns take one more
// product each.  The host diagonalises H and V = Q U for the q smallest
// eigenvalues.  Unlike a single Krylov vector, a block of q vectors spans a
// whole eigenspace of multiplicity up to q.  theta: ascending Ritz values;
// V: device n x q column-major (unit, orthonormal); resid (optional): Ritz
// residuals ||Z v - theta v||, one product each.
static alm_bm_status block_krylov(alm_bm_problem* p, const double* y, int q, int kmax, uint64_t seed,
                                  std::vector<double>& theta, double* V, std::vector<double>* resid, int& m_out,
                                  hipStream_t st) {
  const auto& d = p->d;
  const long n = d.n, ldq = n;
  const int nb = p->lnb, pstride = p->kmax + 1, ld = p->kmax + 1;
  kmax = std::min(kmax, p->kmax);
  const int m = (int)std::min<long>(kmax + 1, n);
  if (q < 1 || q > kMaxBlockQ) return fail(ALM_BM_ERR_INVALID_ARG, "block Lanczos: q must be in 1..8");
  if (kmax < 1 || m < q + 1) return fail(ALM_BM_ERR_INVALID_ARG, "block Lanczos: basis smaller than q + 1");
  double* qsum = (d.j_coef != 0.0) ? &p->sc_api->qsum : nullptr;
  const int cons = d.cons_kind == ALM_BM_CONS_DIAG ? 0 : 1;
  // lw against columns 0..c-1 (two passes; partial ||lw||^2 left in lpart2)
  auto second_pass = [&](int c) {
    launch_dots(n, c, p->Q, ldq, p->lw, p->lpart, pstride, nb, p->lh2, st);
    launch_sub(n, c, p->Q, ldq, p->lh2, p->lw, p->lpart2, nb, st);
  };
  auto normalise_into = [&](int c) -> alm_bm_status {
    launch_fin_sum(p->lpart2, nb, p->lscal, 1, st);
    launch_scale(n, p->lw, p->lscal, p->Q + (long)c * ldq, p->lpart2, nb, qsum, st);
    if (qsum) HIPCHK(hipMemcpyAsync(p->bk_colsum + c, qsum, sizeof(double), hipMemcpyDeviceToDevice, st));
    return ALM_BM_OK;
  };
  auto product = [&](int j) -> alm_bm_status {
    if (qsum) HIPCHK(hipMemcpyAsync(qsum, p->bk_colsum + j, sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_slack_mv(p->C64, cons, p->adj, y, d.trace_coef, d.j_coef, p->sc_api, p->Q + (long)j * ldq, p->lw, st);
    return ALM_BM_OK;
  };
  for (int i = 0; i < q; ++i) {
    launch_rand(n, seed * 1000003ull + (uint64_t)i, p->lw, p->lpart2, nb, st);
    if (i > 0) {
      launch_dots(n, i, p->Q, ldq, p->lw, p->lpart, pstride, nb, p->lh1, st);
      launch_sub(n, i, p->Q, ldq, p->lh1, p->lw, p->lpart2, nb, st);
      second_pass(i);
    }
    STCHK(normalise_into(i));
  }
  for (int c = q; c < m; ++c) {
    const int j = c - q;
    STCHK(product(j));
    launch_dots(n, c, p->Q, ldq, p->lw, p->lpart, pstride, nb, p->lh1, st);
    HIPCHK(hipMemcpyAsync(p->bk_h + (long)j * ld, p->lh1, c * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_sub(n, c, p->Q, ldq, p->lh1, p->lw, p->lpart2, nb, st);
    second_pass(c);
    launch_fin_sum(p->lpart2, nb, p->lscal, 1, st);
    // the new column's norm before scaling: H[c][j] (breakdown test)
    HIPCHK(hipMemcpyAsync(p->bk_h + (long)j * ld + c, p->lscal, sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_scale(n, p->lw, p->lscal, p->Q + (long)c * ldq, p->lpart2, nb, qsum, st);
    if (qsum) HIPCHK(hipMemcpyAsync(p->bk_colsum + c, qsum, sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  for (int j = m - q; j < m; ++j) {
    STCHK(product(j));
    launch_dots(n, m, p->Q, ldq, p->lw, p->lpart, pstride, nb, p->lh1, st);
    HIPCHK(hipMemcpyAsync(p->bk_h + (long)j * ld, p->lh1, m * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  std::vector<double> Hd((size_t)ld * m), cs(m, 0.0);
  HIPCHK(hipMemcpyAsync(Hd.data(), p->bk_h, Hd.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  if (qsum) HIPCHK(hipMemcpyAsync(cs.data(), p->bk_colsum, m * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // the basis ends before the first column whose unnormalised norm vanished
  // (an invariant subspace): later columns are normalised rounding noise
  double hmax = 0.0;
  for (int j = 0; j < m; ++j)
    for (int i = 0; i <= j; ++i) hmax = std::max(hmax, std::fabs(Hd[(size_t)j * ld + i]));
  int mm = m;
  for (int c = q; c < m; ++c) {
    const double beta = Hd[(size_t)(c - q) * ld + c];
    if (!(beta > 1e-12 * std::max(hmax, 1e-300))) {
      mm = c;
      break;
    }
  }
  std::vector<double> Hs((size_t)mm * mm);
  for (int j = 0; j < mm; ++j)
    for (int i = 0; i <= j; ++i) {
      const double h = Hd[(size_t)j * ld + i];
      if (!std::isfinite(h)) return fail(ALM_BM_ERR_NUMERIC, "block Lanczos: NaN/Inf");
      Hs[(size_t)i * mm + j] = Hs[(size_t)j * mm + i] = h;
    }
  std::vector<double> lam, U;
  small_sym_eig(mm, Hs, lam, U);
  std::vector<int> ord(mm);
  for (int k = 0; k < mm; ++k) ord[k] = k;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return lam[a] < lam[b]; });
  const int qv = std::min(q, mm);
  theta.assign(qv, 0.0);
  std::vector<double> coef((size_t)qv * mm);
  for (int k = 0; k < qv; ++k) {
    theta[k] = lam[ord[k]];
    for (int i = 0; i < mm; ++i) coef[(size_t)k * mm + i] = U[(size_t)i * mm + ord[k]];
  }
  HIPCHK(hipMemcpyAsync(p->bk_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, st));
  for (int k = 0; k < qv; ++k)
    launch_combine(n, mm, p->Q, ldq, p->bk_coef + (long)k * mm, V + (long)k * n, p->lpart2, nb, st);
  if (resid) {
    resid->assign(qv, 0.0);
    for (int k = 0; k < qv; ++k) {
      double qs = 0.0;  // 1^T v for the -J term, from the columns' sums
      for (int i = 0; i < mm; ++i) qs += coef[(size_t)k * mm + i] * cs[i];
      if (qsum) HIPCHK(hipMemcpyAsync(qsum, &qs, sizeof(double), hipMemcpyHostToDevice, st));
      launch_slack_mv(p->C64, cons, p->adj, y, d.trace_coef, d.j_coef, p->sc_api, V + (long)k * n, p->lw, st);
      launch_resid(n, p->lw, V + (long)k * n, theta[k], nullptr, p->lpart2, nb, st);
      launch_fin_sum(p->lpart2, nb, p->lscal + 2, 1, st);
      HIPCHK(hipMemcpyAsync(&(*resid)[k], p->lscal + 2, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));  // qs and the result are host values of this iteration
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  m_out = mm;
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_lanczos_block(alm_bm_problem* p, const double* y, int32_t q, int32_t max_iter,
                                             uint64_t seed, double* theta, double* V, double* resid,
                                             int32_t* basis, hipStream_t st) {
  if (!p || !y || !theta) return fail(ALM_BM_ERR_INVALID_ARG, "lanczos_block: null argument");
  if (q < 1 || q > kMaxBlockQ) return fail(ALM_BM_ERR_INVALID_ARG, "lanczos_block: q must be in 1..8");
  if (max_iter < 1 || max_iter > p->kmax)
    return fail(ALM_BM_ERR_INVALID_ARG, "lanczos_block: max_iter must be in 1..lanczos_kmax");
  if (std::min<long>(max_iter + 1, p->d.n) < q + 1)
    return fail(ALM_BM_ERR_INVALID_ARG, "lanczos_block: basis (min(max_iter + 1, n)) must exceed q");
  if (!V && (!p->vblk || q > p->d.rank_block_max))
    return fail(ALM_BM_ERR_INVALID_ARG, "lanczos_block: V is required unless rank_block_max >= q");
  HIPCHK(hipStreamSynchronize(st));
  std::vector<double> th, rs;
  int m = 0;
  STCHK(block_krylov(p, y, q, max_iter, seed, th, V ? V : p->vblk, resid ? &rs : nullptr, m, st));
  for (int k = 0; k < q; ++k) {
    theta[k] = k < (int)th.size() ? th[k] : NAN;
    if (resid) resid[k] = k < (int)rs.size() ? rs[k] : NAN;
  }
  if (basis) *basis = m;
  return ALM_BM_OK;
}

// --------------------------------------------------------------------- KKT

struct KktVals {
  double pinf, dinf, gap, kkt, pobj, dobj;
  double rq;  // <Z(y), RR^T> / ||R||_F^2, an upper bound on lambda_min(Z(y)) (+inf when R = 0)
};

// Rayleigh quotient of X = RR^T for the slack Z(y) = C - A*(y), from the totals
// of an objective pass at (R, y): <Z, X> = <C, X> - y^T A(X) and
// y^T A(X) = b^T y - <y, b - A(X)>.  lambda_min(Z) is at most the
// X-weighted mean of Z's Rayleigh quotients, i.e. this value.
static double slack_rq(double pobj, double dobj, double ybma, double rr) {
  return rr > 0.0 ? (pobj - dobj + ybma) / rr : INFINITY;
}

// Relative KKT terms of Sec. 6 at (RR^T, y).  lam is the caller's estimate of
// lambda_min(Z(y)) (a Ritz value, so an upper bound); the dual infeasibility
// uses min(lam, rq), the tighter of two upper bounds.
static void kkt_terms(double pobj, double dobj, double pinf, double lam, double rq, double cnorm, KktVals& k) {
  k.pobj = pobj;
  k.dobj = dobj;
  k.pinf = pinf;
  k.rq = rq;
  k.dinf = std::fabs(std::min(0.0, std::min(lam, rq))) / (1.0 + cnorm);
  k.gap = std::fabs(pobj - dobj) / (1.0 + std::fabs(pobj) + std::fabs(dobj));
  k.kkt = std::max(k.pinf, std::max(k.dinf, k.gap));
}

// pobj and pinf at R, dobj at y (device y), lambda_min given.  tighten: the
// dual term takes min(lam, rq) (inside the solve); otherwise lam as given
// (alm_bm_kkt, the plain Sec. 6 measure for a supplied lambda_min).
template <typename T>
static alm_bm_status kkt_eval(alm_bm_problem* p, int r, const T* R, const double* y, double lam, KktVals& k,
                              hipStream_t st, bool tighten = true) {
  enqueue_objgrad<T>(p, r, R, y, 0.0, nullptr, p->Av, p->sc_api, 0, nullptr, st);
  launch_dual(p->d.m, p->Av, p->d.b, y, nullptr, 0.0, p->part_vec, p->sc_api, p->bnorm, nullptr, st);
  HIPCHK(hipMemcpyAsync(p->sc_host, p->sc_api, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  const DevScalars& s = *p->sc_host;
  const double rq = slack_rq(s.tot[P_C0], s.dobj, s.tot[P_YBMA], s.tot[P_RR]);
  kkt_terms(s.tot[P_C0], s.dobj, s.pinf, lam, tighten ? rq : INFINITY, p->cnorm, k);
  k.rq = rq;
  return ALM_BM_OK;
}

// A Ritz pair (theta, residual) bounds an eigenvalue of the slack to
// [theta - resid, theta + resid]; taken as the bottom of the spectrum (what a
// Krylov space from a random start finds first), it certifies the dual
// infeasibility term when even the low end theta - resid meets the tolerance:
// resid - theta <= dtol = eps (1 + ||C||_F).  A Ritz value above the Rayleigh
// quotient of X (plus ltol) belongs to an eigenvalue other than the smallest
// and certifies nothing.  Near an optimum the bottom of the spectrum is a
// cluster of about rank-many eigenvalues near zero, where the Ritz residual
// stalls far above its own tolerance while theta itself is tiny; this test
// accepts such a pair when its whole interval is dual feasible to dtol.
static bool lanczos_certifies(double theta, double resid, double ltol, double rq, double dtol) {
  return std::isfinite(theta) && std::isfinite(resid) && theta <= rq + ltol && resid - theta <= dtol;
}

extern "C" alm_bm_status alm_bm_kkt(alm_bm_problem* p, int32_t r, const void* R, const double* y, double lam_min,
                                    double* kkt_out, hipStream_t st) {
  if (!p || !R || !y || !kkt_out) return fail(ALM_BM_ERR_INVALID_ARG, "kkt: null argument");
  STCHK(check_r(p, r));
  KktVals k{};
  alm_bm_status s = with_storage(p->d.precision, [&]<typename T>() {
    return kkt_eval<T>(p, r, static_cast<const T*>(R), y, lam_min, k, st, false);
  });
  if (s < 0) return s;
  kkt_out[0] = k.pinf;
  kkt_out[1] = k.dinf;
  kkt_out[2] = k.gap;
  kkt_out[3] = k.kkt;
  kkt_out[4] = k.pobj;
  kkt_out[5] = k.dobj;
  return ALM_BM_OK;
}

// --------------------------------------------------------------------- solve

namespace {

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int r = -1;
  int refresh = -1;
  int lb_m = -1;
  const void* R = nullptr;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    r = -1;
    R = nullptr;
  }
  ~GraphCache() { reset(); }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int bp_rank_cap(long m) {
  long r = (long)((std::sqrt(8.0 * (double)m + 1.0) - 1.0) / 2.0);
  while ((r + 1) * (r + 2) / 2 <= m) ++r;
  while (r > 0 && r * (r + 1) / 2 > m) --r;
  return (int)r;
}

}  // namespace

template <typename T>
static alm_bm_status inner_solve(alm_bm_problem* p, int r, T* R, const double* y, double sigma, double tol,
                                 const alm_bm_options& o, GraphCache& gc, hipStream_t st, int& iters, int& flag) {
  T* G = static_cast<T*>(p->G);
  const int refresh = o.refresh_every > 0 ? o.refresh_every : default_refresh(sizeof(T) == 8 ? ALM_BM_F64
                                                                  : (sizeof(T) == 4 ? ALM_BM_F32 : ALM_BM_BF16));
  launch_inner_reset(p->sc_solve, tol, o.max_inner, (int)o.step_rule, o.eta_fixed, st);
  if (p->lb_m > 0) launch_lbfgs_reset(p->lbs, p->lb_m, st);  // each subproblem starts with an empty memory
  const int U = std::max(0, o.graph_unroll);
  int32_t hflag = 0;
  const int max_launch = o.max_inner + 2;
  int launched = 0;
  while (true) {
    if (U > 0) {
      if (gc.r != r || gc.R != (const void*)R || gc.refresh != refresh || gc.lb_m != p->lb_m) {
        gc.reset();
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int u = 0; u < U; ++u) enqueue_inner_step<T>(p, r, R, y, sigma, G, refresh, st);
        HIPCHK(hipStreamEndCapture(st, &gc.graph));
        HIPCHK(hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0));
        gc.r = r;
        gc.R = R;
        gc.refresh = refresh;
        gc.lb_m = p->lb_m;
      }
      HIPCHK(hipGraphLaunch(gc.exec, st));
      launched += U;
    } else {
      enqueue_inner_step<T>(p, r, R, y, sigma, G, refresh, st);
      launched += 1;
    }
    HIPCHK(hipMemcpyAsync(&p->sc_host->flag, &p->sc_solve->flag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    hflag = p->sc_host->flag;
    if (hflag != 0) break;
    if (launched > max_launch + U) return fail(ALM_BM_ERR_HIP, "inner loop did not reach its stop flag");
  }
  HIPCHK(hipGetLastError());
  iters = p->sc_host->iter;
  flag = hflag;
  return ALM_BM_OK;
}

// Row width of the factor inside a solve: the next tile width (4, 8, 16, 32, ...)
// at or above the rank, so that rows stay aligned and every kernel takes its
// full-tile path; the padding columns hold zeros, which every map of the method
// keeps at zero, and a rank step fills the first of them.
static int pad_width(int r, int r_max) {
  int w = 4;
  while (w < r) w *= 2;
  return std::min(w, std::max(r, r_max));
}

// R (n x r, row stride r) <-> the same factor at row stride w, through the
// handle's n x r_max scratch.
template <typename T>
static alm_bm_status restride(alm_bm_problem* p, T* R, int ss, int nc, int rd, hipStream_t st) {
  if (ss == rd && nc == rd) return ALM_BM_OK;
  T* Rt = static_cast<T*>(p->Rtmp);
  launch_relayout<T>(p->d.n, ss, nc, rd, R, Rt, nullptr, 0.0, st);
  HIPCHK(hipMemcpyAsync(R, Rt, (size_t)p->d.n * rd * sizeof(T), hipMemcpyDeviceToDevice, st));
  return ALM_BM_OK;
}

// Penalty quadratic form of A(V S V^T) over the pairs a <= b of q orthonormal
// directions V (device n x q, column-major): M4[pair(a,b), pair(c,d)] = sum over
// constraint rows of A_i(v_a v_b^T) A_i(v_c v_d^T), edge rows weighted by
// edge_w.  Fourth moments per block from k_gram4 / k_gram4_edges, summed on the
// host in block order; the trace row adds c_tr^2 [a = b][c = d].
static alm_bm_status block_moments(alm_bm_problem* p, int q, const double* V, double edge_w, std::vector<double>& M4,
                                   hipStream_t st) {
  const auto& d = p->d;
  const int np = q * (q + 1) / 2, ne = np * (np + 1) / 2;
  const bool edges = d.cons_kind != ALM_BM_CONS_DIAG;
  if (edges) launch_gram4_edges(d.n_edges, d.n, q, d.edge_i, d.edge_j, V, p->gpart, p->lnb, st);
  else launch_gram4(d.n, q, V, p->gpart, p->lnb, st);
  std::vector<double> gp((size_t)p->lnb * ne);
  HIPCHK(hipMemcpyAsync(gp.data(), p->gpart, gp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  M4.assign((size_t)np * np, 0.0);
  for (int e = 0, p1 = 0, p2 = 0; e < ne; ++e) {
    double s = 0.0;
    for (int b = 0; b < p->lnb; ++b) s += gp[(size_t)b * ne + e];
    M4[(size_t)p1 * np + p2] = M4[(size_t)p2 * np + p1] = (edges ? edge_w : 1.0) * s;
    if (++p2 == np) p2 = ++p1;
  }
  if (edges && d.trace_coef != 0.0) {
    // trace row: c_tr tr(V S V^T) = c_tr tr(S) for orthonormal V
    for (int a0 = 0; a0 < q; ++a0)
      for (int c0 = 0; c0 < q; ++c0) {
        const int pa = a0 * q - a0 * (a0 - 1) / 2, pc = c0 * q - c0 * (c0 - 1) / 2;  // index of (a, a), (c, c)
        M4[(size_t)pa * np + pc] += d.trace_coef * d.trace_coef;
      }
  }
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_block_moments(alm_bm_problem* p, int32_t q, const double* V, double edge_weight,
                                              double* M4, hipStream_t st) {
  if (!p || !V || !M4) return fail(ALM_BM_ERR_INVALID_ARG, "block_moments: null argument");
  if (q < 1 || q > p->d.rank_block_max || !p->gpart)
    return fail(ALM_BM_ERR_INVALID_ARG, "block_moments: q must be in 1..rank_block_max of the handle");
  if (!(edge_weight >= 0.0)) return fail(ALM_BM_ERR_INVALID_ARG, "block_moments: edge_weight must be >= 0");
  std::vector<double> out;
  STCHK(block_moments(p, q, V, edge_weight, out, st));
  std::copy(out.begin(), out.end(), M4);
  return ALM_BM_OK;
}

// Block rank step (Alg. 1 with several directions): the
// smallest Ritz pairs below -tau_rank of a full Lanczos pass on Z(w) from a
// random start give V (n x qv, orthonormal, V^T Z V = diag(theta)); k_gram4
// (rows, DIAG) or k_gram4_edges (edge rows, weighted by rho, plus the trace
// row's c_tr^2 tr(S)^2) gives the penalty's quadratic form, the host solves
// the qv x qv PSD subproblem, and the columns of V S^{1/2} are appended to R.
template <typename T>
static alm_bm_status block_rank_step(alm_bm_problem* p, T* R, int& r, int& w, int r_cap, int rank_block,
                                     double sigma, int kmax, double tau_rank, uint64_t seed, GraphCache& gc,
                                     int& added, hipStream_t st) {
  const auto& d = p->d;
  const long n = d.n;
  added = 0;
  const int q = std::min(rank_block, r_cap - r);
  if (q < 1) return ALM_BM_OK;
  if (!p->vblk || rank_block > d.rank_block_max)
    return fail(ALM_BM_ERR_INVALID_ARG, "block rank step: rank_block exceeds the handle's rank_block_max");
  // the q smallest Ritz pairs of a block Krylov space of block size q (a
  // repeated eigenvalue contributes its whole eigenspace), V into vblk
  const int qk = (int)std::min<long>(q, std::min<long>(std::min(kmax, p->kmax) + 1, n) - 1);
  if (qk < 1) return ALM_BM_OK;
  std::vector<double> thb;
  int m = 0;
  STCHK(block_krylov(p, p->ybuf, qk, kmax, seed, thb, p->vblk, nullptr, m, st));
  int qv = 0;
  while (qv < (int)thb.size() && thb[qv] < -tau_rank) ++qv;
  if (qv == 0) return ALM_BM_OK;
  const std::vector<double> th(thb.begin(), thb.begin() + qv);
  const int np = qv * (qv + 1) / 2;
  std::vector<double> M4;
  STCHK(block_moments(p, qv, p->vblk, p->rho, M4, st));
  const std::vector<double> S = block_subproblem(qv, th, M4, np, sigma);
  std::vector<double> lam, U;
  small_sym_eig(qv, S, lam, U);
  double lmax = 0.0;
  for (double v : lam) lmax = std::max(lmax, v);
  std::vector<double> coef;
  for (int k = 0; k < qv && r + added < r_cap; ++k) {
    if (!(lam[k] > 1e-14 * std::max(lmax, 1e-300))) continue;
    for (int i = 0; i < qv; ++i) coef.push_back(U[i * qv + k] * std::sqrt(lam[k]));
    ++added;
  }
  if (added == 0) return ALM_BM_OK;
  HIPCHK(hipMemcpyAsync(p->ycoef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, st));
  for (int j = 0; j < added; ++j) {
    launch_combine(n, qv, p->vblk, n, p->ycoef + (long)j * qv, p->lw, p->lpart2, p->lnb, st);
    if (r + 1 <= w) {
      launch_set_column<T>(n, w, r, R, p->lw, 1.0, st);
    } else {
      const int w2 = pad_width(r + 1, d.r_max);
      T* Rt = static_cast<T*>(p->Rtmp);
      launch_relayout<T>(n, w, r, w2, R, Rt, p->lw, 1.0, st);
      HIPCHK(hipMemcpyAsync(R, Rt, (size_t)n * w2 * sizeof(T), hipMemcpyDeviceToDevice, st));
      w = w2;
      gc.reset();
    }
    r += 1;
  }
  HIPCHK(hipStreamSynchronize(st));
  return ALM_BM_OK;
}

template <typename T>
static alm_bm_status solve_impl(alm_bm_problem* p, const alm_bm_options& o, T* R, double* y, hipStream_t st,
                                int& r, int& w, int k_start, int& k_done,
                                bool stop_on_stall, bool& stalled, double t0, double& pinf_prev, double& tol_prev,
                                double& sigma, alm_bm_result& acc) {
  const auto& d = p->d;
  const long n = d.n;
  const double tau_rank = o.tau_rank > 0.0 ? o.tau_rank : o.eps_kkt * (1.0 + p->cnorm);
  int r_cap = std::min<int>(d.r_max, bp_rank_cap(d.m));
  if (o.r_cap > 0) r_cap = std::min(r_cap, o.r_cap);
  const int kmax = o.lanczos_kmax > 0 ? std::min(o.lanczos_kmax, p->kmax) : p->kmax;
  const double ltol = o.lanczos_tol_rel * o.eps_kkt * (1.0 + p->cnorm);
  GraphCache gc;
  stalled = false;
  std::vector<double> pinf_hist;
  for (int k = k_start; k < o.max_outer; ++k) {
    const double pinf_last = pinf_prev;  // of the previous outer iteration (inf at the start)
    const double tol = std::max(o.eps_kkt / 10.0, std::min(o.inner_tol_scale, std::min(pinf_prev, o.inner_tol_decay * tol_prev)));
    tol_prev = tol;
    acc.inner_tol = tol;
    int iters = 0, flag = 0;
    STCHK(inner_solve<T>(p, w, R, y, sigma, tol, o, gc, st, iters, flag));
    acc.inner_total += iters;
    // w = y - sigma (A(RR^T) - b) into ybuf (Av is current: the last pass ran at the final R)
    launch_dual(d.m, p->Av, d.b, y, p->ybuf, sigma, p->part_vec, p->sc_solve, p->bnorm, nullptr, st,
                sigma * p->rho);
    LanczosOut lo;
    const double tl = now_s();
    STCHK(lanczos_run(p, p->ybuf, kmax, ltol, o.seed * 1000003ull + (uint64_t)k, p->lv, lo, st,
                      o.lanczos_restarts));
    acc.time_lanczos_s += now_s() - tl;
    // KKT of the point as it stands (the final one unless a rank step follows)
    KktVals kv{};
    STCHK(kkt_eval<T>(p, w, R, p->ybuf, lo.theta, kv, st));
    // The rank test of Alg. 1 asks for theta < -tau.  A point that meets the KKT
    // tolerance but whose Ritz interval reaches below -dtol although the
    // residual alone would allow a certificate (resid < dtol) has negative
    // curvature that blocks the certificate while staying above -tau; it
    // takes the rank step too, or the solve would repeat the same outer
    // iteration until max_outer.
    const double dtol = o.eps_kkt * (1.0 + p->cnorm);
    const bool blocked = kv.kkt <= o.eps_kkt && lo.resid < dtol && lo.resid - lo.theta > dtol;
    const double tau_k = blocked ? 0.0 : tau_rank;
    bool expanded = false;
    const bool gate = (flag == 1) || !o.expand_needs_inner;
    if (o.rank_policy == ALM_BM_RANK_ADAPT && gate && lo.theta < -tau_k && r < r_cap && o.rank_block > 1) {
      int added = 0;
      STCHK(block_rank_step<T>(p, R, r, w, r_cap, o.rank_block, sigma, kmax, tau_k,
                               o.seed * 1000003ull + (uint64_t)k + 3333333ull, gc, added, st));
      if (added > 0) {
        expanded = true;
        acc.expansions += 1;
        enqueue_objgrad<T>(p, w, R, y, sigma, nullptr, p->Av, p->sc_api, 0, nullptr, st);
        launch_dual(d.m, p->Av, d.b, y, p->ybuf, sigma, p->part_vec, p->sc_solve, p->bnorm, nullptr, st,
                    sigma * p->rho);
      }
    } else if (o.rank_policy == ALM_BM_RANK_ADAPT && gate && lo.theta < -tau_k && r < r_cap) {
      // ||A(v v^T)||^2 for the unit Ritz vector
      launch_quartic_norm(n, d.cons_kind == ALM_BM_CONS_DIAG ? 0 : 1, p->adj, p->lv, p->lpart2, p->lnb, st);
      launch_fin_sum(p->lpart2, p->lnb, p->lscal + 3, 0, st);
      double q4 = 0.0;
      HIPCHK(hipMemcpyAsync(&q4, p->lscal + 3, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      // curvature sum_i sigma_i a_i(v v^T)^2 / sigma of the rank-one step (edge rows weighted by rho)
      if (d.cons_kind != ALM_BM_CONS_DIAG) q4 = p->rho * q4 + d.trace_coef * d.trace_coef;
      if (q4 > 0.0) {
        const double s = std::max(0.0, -lo.theta / (sigma * q4));
        if (r + 1 <= w) {
          launch_set_column<T>(n, w, r, R, p->lv, std::sqrt(s), st);
        } else {
          const int w2 = pad_width(r + 1, d.r_max);
          T* Rt = static_cast<T*>(p->Rtmp);
          launch_relayout<T>(n, w, r, w2, R, Rt, p->lv, std::sqrt(s), st);
          HIPCHK(hipMemcpyAsync(R, Rt, (size_t)n * w2 * sizeof(T), hipMemcpyDeviceToDevice, st));
          w = w2;
          gc.reset();
        }
        r += 1;
        expanded = true;
        acc.expansions += 1;
        enqueue_objgrad<T>(p, w, R, y, sigma, nullptr, p->Av, p->sc_api, 0, nullptr, st);
        launch_dual(d.m, p->Av, d.b, y, p->ybuf, sigma, p->part_vec, p->sc_solve, p->bnorm, nullptr, st,
                    sigma * p->rho);
      }
    }
    HIPCHK(hipMemcpyAsync(y, p->ybuf, d.m * sizeof(double), hipMemcpyDeviceToDevice, st));
    double lam = lo.theta, lres = lo.resid;
    if (expanded) {
      LanczosOut l2;
      const double tl2 = now_s();
      STCHK(lanczos_run(p, y, kmax, ltol, o.seed * 1000003ull + (uint64_t)k + 7777777ull, p->lv, l2, st,
                        o.lanczos_restarts));
      acc.time_lanczos_s += now_s() - tl2;
      lam = l2.theta;
      lres = l2.resid;
      STCHK(kkt_eval<T>(p, w, R, y, lam, kv, st));
    }
    if (p->sc_host->numeric_error) return fail(ALM_BM_ERR_NUMERIC, "solve: NaN/Inf in objective or step");
    HIPCHK(hipMemcpyAsync(p->sc_host, p->sc_solve, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (p->sc_host->numeric_error) return fail(ALM_BM_ERR_NUMERIC, "solve: NaN/Inf in objective or step");
    if (!std::isfinite(kv.kkt)) return fail(ALM_BM_ERR_NUMERIC, "solve: non-finite KKT");
    acc.outer = k + 1;
    acc.rank = r;
    acc.pobj = kv.pobj;
    acc.dobj = kv.dobj;
    acc.pinf = kv.pinf;
    acc.dinf = kv.dinf;
    acc.gap = kv.gap;
    acc.kkt = kv.kkt;
    acc.lam_min = std::min(lam, kv.rq);
    acc.lanczos_resid = lres;
    pinf_prev = kv.pinf;
    k_done = k + 1;
    const bool cert = lanczos_certifies(lam, lres, ltol, kv.rq, o.eps_kkt * (1.0 + p->cnorm));
    if (o.verbose)
      std::fprintf(stderr,
                   "[almbm] k=%d inner=%d flag=%d r=%d theta=%.3e rq=%.3e lres=%.2e%s lanczos=%d pinf=%.3e "
                   "dinf=%.3e gap=%.3e pobj=%.10e sigma=%.3e t=%.2fs\n",
                   k, iters, flag, r, lam, kv.rq, lres, cert ? "" : "(uncertified)", lo.iters, kv.pinf, kv.dinf,
                   kv.gap, kv.pobj, sigma, now_s() - t0);
    if (kv.kkt <= o.eps_kkt && cert) return ALM_BM_OK;
    // penalty schedule: raise sigma when the infeasibility did not fall enough
    if (o.sigma_growth > 1.0 && kv.pinf > o.pinf_reduction * pinf_last && sigma < o.sigma_max) {
      sigma = std::min(o.sigma_max, sigma * o.sigma_growth);
      acc.sigma_final = sigma;
      acc.sigma_increases += 1;
      gc.reset();  // the captured inner loop holds sigma as a kernel argument
    }
    if (o.time_limit_s > 0.0 && now_s() - t0 > o.time_limit_s) return ALM_BM_NOT_CONVERGED;
    if (stop_on_stall) {
      // storage-precision floor: primal infeasibility no longer falls by 2x over 3 outer iterations
      pinf_hist.push_back(kv.pinf);
      const size_t h = pinf_hist.size();
      if (h >= 4 && pinf_hist[h - 1] > 0.5 * pinf_hist[h - 4] && kv.pinf > o.eps_kkt) {
        stalled = true;
        return ALM_BM_NOT_CONVERGED;
      }
    }
  }
  return ALM_BM_NOT_CONVERGED;
}

extern "C" alm_bm_status alm_bm_inner_solve(alm_bm_problem* p, const alm_bm_options* opts, int32_t r, void* R,
                                            const double* y, double tol, int32_t max_steps, int32_t* steps_done,
                                            int32_t* stop_flag, double* f_last, hipStream_t st_user) {
  if (!p || !R || !y) return fail(ALM_BM_ERR_INVALID_ARG, "inner_solve: null argument");
  STCHK(check_r(p, r));
  if (max_steps < 0) return fail(ALM_BM_ERR_INVALID_ARG, "inner_solve: max_steps < 0");
  alm_bm_options o;
  if (opts) o = *opts;
  else alm_bm_default_options(&o);
  if (!(o.sigma > 0.0)) return fail(ALM_BM_ERR_INVALID_ARG, "inner_solve: sigma must be positive");
  o.max_inner = max_steps;
  if (o.sigma_edges < 0.0) return fail(ALM_BM_ERR_INVALID_ARG, "inner_solve: sigma_edges must be >= 0");
  HIPCHK(hipStreamSynchronize(st_user));
  hipStream_t st = p->ss;
  struct RhoScope {
    alm_bm_problem* p;
    ~RhoScope() { p->rho = 1.0; }
  } rho_scope{p};
  p->rho = (p->d.cons_kind != ALM_BM_CONS_DIAG && o.sigma_edges > 0.0) ? o.sigma_edges / o.sigma : 1.0;
  int lb_m = 0;
  STCHK(check_inner(p, o, lb_m));
  InnerScope inner_scope(p, lb_m);
  int iters = 0, flag = 0;
  GraphCache gc;
  alm_bm_status s = with_storage(p->d.precision, [&]<typename T>() {
    return inner_solve<T>(p, r, static_cast<T*>(R), y, o.sigma, tol, o, gc, st, iters, flag);
  });
  if (s < 0) return s;
  HIPCHK(hipMemcpyAsync(p->sc_host, p->sc_solve, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (steps_done) *steps_done = iters;
  if (stop_flag) *stop_flag = flag;
  if (f_last) *f_last = p->sc_host->f;
  if (p->sc_host->numeric_error) return fail(ALM_BM_ERR_NUMERIC, "inner_solve: NaN/Inf");
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_solve(alm_bm_problem* p, const alm_bm_options* opts, void* R, int32_t* r_io,
                                      double* y, alm_bm_result* out, hipStream_t st_user) {
  if (!p || !R || !r_io || !y) return fail(ALM_BM_ERR_INVALID_ARG, "solve: null argument");
  STCHK(check_r(p, *r_io));
  alm_bm_options o;
  if (opts) o = *opts;
  else alm_bm_default_options(&o);
  if (!(o.sigma > 0.0) || !(o.eps_kkt > 0.0) || o.max_outer < 1 || o.max_inner < 1)
    return fail(ALM_BM_ERR_INVALID_ARG, "solve: sigma, eps_kkt, max_outer and max_inner must be positive");
  if (p->kmax < 1) return fail(ALM_BM_ERR_INVALID_ARG, "solve: the handle has no Lanczos workspace");
  if (o.sigma_edges < 0.0) return fail(ALM_BM_ERR_INVALID_ARG, "solve: sigma_edges must be >= 0");
  if (!(o.sigma_growth >= 1.0) || !(o.sigma_max >= o.sigma) || !(o.pinf_reduction > 0.0 && o.pinf_reduction <= 1.0))
    return fail(ALM_BM_ERR_INVALID_ARG, "solve: need sigma_growth >= 1, sigma_max >= sigma, 0 < pinf_reduction <= 1");
  if (o.resume_outer < 0 || o.resume_outer >= o.max_outer)
    return fail(ALM_BM_ERR_INVALID_ARG, "solve: resume_outer must be in 0..max_outer-1");
  if (o.rank_block < 1 || o.rank_block > std::max(1, p->d.rank_block_max))
    return fail(ALM_BM_ERR_INVALID_ARG, "solve: rank_block must be in 1..rank_block_max of the handle (" +
                                            std::to_string(std::max(1, p->d.rank_block_max)) + ")");
  int lb_m = 0;
  STCHK(check_inner(p, o, lb_m));
  HIPCHK(hipStreamSynchronize(st_user));
  hipStream_t st = p->ss;
  InnerScope inner_scope(p, lb_m);
  // a NaN seen by an earlier call must not fail this one
  HIPCHK(hipMemsetAsync(&p->sc_api->numeric_error, 0, sizeof(int32_t), st));
  // penalty of the edge rows relative to sigma, for the length of this solve
  struct RhoScope {
    alm_bm_problem* p;
    ~RhoScope() { p->rho = 1.0; }
  } rho_scope{p};
  p->rho = (p->d.cons_kind != ALM_BM_CONS_DIAG && o.sigma_edges > 0.0) ? o.sigma_edges / o.sigma : 1.0;
  const double t0 = now_s();
  alm_bm_result acc{};
  acc.promoted_at_outer = -1;
  int r = *r_io;
  int w = pad_width(r, p->d.r_max);
  // resume: the outer index (Lanczos seeds) and the tolerance recurrence of a
  // stopped solve, so that stopping and resuming repeats the uninterrupted solve
  const int k0 = o.resume_outer;
  int k_done = k0;
  double pinf_prev = o.resume_pinf > 0.0 ? o.resume_pinf : INFINITY;
  double tol_prev = o.resume_inner_tol > 0.0 ? o.resume_inner_tol : INFINITY;
  double sigma = o.sigma;
  acc.sigma_final = sigma;
  bool stalled = false;
  alm_bm_status s;
  p->ladder_r = 0;
  if (p->d.precision == ALM_BM_BF16 && o.bf16_promote) {
    bf16* Rb = static_cast<bf16*>(R);
    STCHK(restride<bf16>(p, Rb, r, r, w, st));
    s = solve_impl<bf16>(p, o, Rb, y, st, r, w, k0, k_done, true, stalled, t0, pinf_prev, tol_prev, sigma, acc);
    if (s >= 0 && stalled) {
      // precision ladder: continue with float storage (the float cost copy is resident)
      const long n = p->d.n;
      float* Rf = static_cast<float*>(p->R32);
      launch_convert<bf16, float>((long)n * w, Rb, Rf, st);
      void* Gsave = p->G;
      void* Rtsave = p->Rtmp;
      p->G = p->G32;
      p->Rtmp = p->Rt32;
      const double tp = now_s();
      acc.promoted_at_outer = k_done;
      s = solve_impl<float>(p, o, Rf, y, st, r, w, k_done, k_done, false, stalled, t0, pinf_prev, tol_prev, sigma, acc);
      alm_bm_status s2 = restride<float>(p, Rf, w, r, r, st);
      p->G = Gsave;
      p->Rtmp = Rtsave;
      acc.time_promoted_s = now_s() - tp;
      STCHK(s2);
      launch_convert<float, bf16>((long)n * r, Rf, Rb, st);
      HIPCHK(hipStreamSynchronize(st));
      if (s < 0) return s;
      p->ladder_r = r;  // the certified point stays in R32 (alm_bm_ladder_factor)
    } else {
      STCHK(restride<bf16>(p, Rb, w, r, r, st));
      if (s < 0) return s;
    }
  } else {
    s = with_storage(p->d.precision, [&]<typename T>() {
      T* Rt = static_cast<T*>(R);
      alm_bm_status s1 = restride<T>(p, Rt, r, r, w, st);
      if (s1 < 0) return s1;
      s1 = solve_impl<T>(p, o, Rt, y, st, r, w, k0, k_done, false, stalled, t0, pinf_prev, tol_prev, sigma, acc);
      const alm_bm_status s2 = restride<T>(p, Rt, w, r, r, st);
      return s1 < 0 ? s1 : (s2 < 0 ? s2 : s1);
    });
    if (s < 0) return s;
  }
  HIPCHK(hipStreamSynchronize(st));
  *r_io = r;
  acc.rank = r;
  acc.time_s = now_s() - t0;
  if (out) *out = acc;
  return s;
}

extern "C" alm_bm_status alm_bm_ladder_factor(alm_bm_problem* p, int32_t r, float* R, hipStream_t st) {
  if (!p || !R) return fail(ALM_BM_ERR_INVALID_ARG, "ladder_factor: null argument");
  if (p->d.precision != ALM_BM_BF16 || p->ladder_r <= 0)
    return fail(ALM_BM_ERR_INVALID_ARG, "ladder_factor: the last solve did not switch to float storage");
  if (r != p->ladder_r) return fail(ALM_BM_ERR_INVALID_ARG, "ladder_factor: r differs from the solve's rank");
  HIPCHK(hipMemcpyAsync(R, p->R32, (size_t)p->d.n * r * sizeof(float), hipMemcpyDeviceToDevice, st));
  return ALM_BM_OK;
}

// ===================================================================== batched solves

struct alm_bm_batch {
  alm_bm_problem* p = nullptr;      // the concatenated super-problem (owns workspace)
  int count = 0;
  int rs = 0;                       // rank stride
  std::vector<int64_t> off;         // count + 1 row offsets
  std::vector<double> cnorm;        // per instance ||C||_F
  std::vector<int> kmax;            // per instance Lanczos basis limit (<= handle kmax)
  std::vector<void*> own;           // device arrays owned by the batch
  double* bnorm_dev = nullptr;      // per instance ||b||
  int32_t* flags_dev = nullptr;     // 2 * count
  double* tols_dev = nullptr;       // count
  int32_t* active_dev = nullptr;    // count
  int32_t* col_dev = nullptr;       // count
  double* scale_dev = nullptr;      // count
  double* thetas_dev = nullptr;     // count
  // Inside a solve every instance keeps its factor at its own padded width
  // w_q (pad_width of its rank) in its region [off_q rs, (off_q + n_q) rs):
  // row i at xbase_q + i w_q.  The row kernels run once per distinct width
  // over the blocks of the active instances of that width (launch tables).
  static constexpr int kNC = 8;
  int32_t* c_inst[kNC] = {};
  int64_t* c_lo[kNC] = {};
  int64_t* c_hi[kNC] = {};
  int32_t* c_gid[kNC] = {};
  int c_nb[kNC] = {};
  int c_w[kNC] = {};
  int c_var[kNC] = {};              // tile variant of each class (from wvar)
  int nclass = 0;
  std::map<int, int> wvar;          // width -> tile variant chosen by alm_bm_batch_autotune
  int32_t* l_inst = nullptr;        // blocks of the instances a Lanczos pass still runs
  int64_t* l_lo = nullptr;
  int64_t* l_hi = nullptr;
  int32_t* l_gid = nullptr;
  int32_t* lm_dev = nullptr;        // count: Lanczos basis size of each instance's pass
  std::vector<int32_t> hl_inst, hl_gid;  // host side of the Lanczos table (kept until uploaded)
  std::vector<int64_t> hl_lo, hl_hi;
  int64_t* xbase_dev = nullptr;     // count
  int64_t* ob_dev = nullptr;        // count: re-layout arguments
  int32_t* os_dev = nullptr;
  int64_t* nbase_dev = nullptr;
  int32_t* ns_dev = nullptr;
  int32_t* nc_dev = nullptr;
  std::vector<int32_t> h_iblo, h_ibhi;  // host copy of the block table
  std::vector<int64_t> h_lo, h_hi;
};

static alm_bm_status balloc(alm_bm_batch* b, void** out, size_t bytes) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) return fail(ALM_BM_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  b->own.push_back(*out);
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_batch_destroy(alm_bm_batch* b) {
  if (!b) return ALM_BM_OK;
  (void)hipDeviceSynchronize();
  if (b->p) alm_bm_destroy(b->p);
  for (void* a : b->own) (void)hipFree(a);
  delete b;
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_batch_offsets(const alm_bm_batch* b, int64_t* offsets) {
  if (!b || !offsets) return fail(ALM_BM_ERR_INVALID_ARG, "batch_offsets: null argument");
  for (int q = 0; q <= b->count; ++q) offsets[q] = b->off[q];
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_batch_create(int32_t count, const alm_bm_problem_desc* descs, int32_t rank_stride,
                                             hipStream_t st, alm_bm_batch** out) {
  if (!descs || !out || count < 1 || count > 4096) return fail(ALM_BM_ERR_INVALID_ARG, "batch_create: bad arguments");
  if (rank_stride < 1 || rank_stride > kMaxR) return fail(ALM_BM_ERR_INVALID_ARG, "batch_create: rank_stride in 1..128");
  *out = nullptr;
  const alm_bm_precision prec = descs[0].precision;
  long N = 0, NNZ = 0;
  int kmax_all = 0, lbm_all = 0;
  for (int q = 0; q < count; ++q) {
    const auto& d = descs[q];
    if (d.cons_kind != ALM_BM_CONS_DIAG || d.m != d.n || d.j_coef != 0.0)
      return fail(ALM_BM_ERR_UNSUPPORTED, "batch_create: DIAG family (m = n, no -J term) only");
    if (d.precision != prec) return fail(ALM_BM_ERR_INVALID_ARG, "batch_create: one precision for all instances");
    if (d.n <= 0 || !d.b || (d.nnz > 0 && (!d.col_idx || !d.val || (d.ell_width == 0 && !d.row_ptr))))
      return fail(ALM_BM_ERR_INVALID_ARG, "batch_create: instance " + std::to_string(q) + " malformed");
    N += d.n;
    NNZ += d.nnz;
    kmax_all = std::max(kmax_all, d.lanczos_kmax);
    if (d.lbfgs_memory_max < 0 || d.lbfgs_memory_max > kMaxLbfgs)
      return fail(ALM_BM_ERR_INVALID_ARG, "batch_create: lbfgs_memory_max must be in 0..8");
    lbm_all = std::max(lbm_all, d.lbfgs_memory_max);
  }
  if (N > INT32_MAX || NNZ > INT32_MAX) return fail(ALM_BM_ERR_UNSUPPORTED, "batch_create: totals exceed int32");
  if (kmax_all < 1) return fail(ALM_BM_ERR_INVALID_ARG, "batch_create: lanczos_kmax must be >= 1");
  HIPCHK(hipStreamSynchronize(st));
  alm_bm_batch* b = new alm_bm_batch();
  b->count = count;
  b->rs = rank_stride;
  auto bail = [&](alm_bm_status s) {
    alm_bm_batch_destroy(b);
    return s;
  };
#define BK(x)                          \
  do {                                 \
    alm_bm_status s_ = (x);            \
    if (s_ < 0) return bail(s_);       \
  } while (0)
#define BH(x)                                                                                          \
  do {                                                                                                 \
    hipError_t e_ = (x);                                                                               \
    if (e_ != hipSuccess) return bail(fail(ALM_BM_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_))); \
  } while (0)
  // ---- concatenate on the host (one round trip at set-up)
  std::vector<int32_t> rp(N + 1), ci(std::max<long>(1, NNZ));
  std::vector<double> cv(std::max<long>(1, NNZ)), dg(N, 0.0), bb(N);
  b->off.assign(count + 1, 0);
  b->cnorm.assign(count, 0.0);
  b->kmax.assign(count, 0);
  std::vector<double> bnorm(count, 0.0);
  long ro = 0, ko = 0;
  rp[0] = 0;
  for (int q = 0; q < count; ++q) {
    const auto& d = descs[q];
    const long n = d.n;
    b->off[q] = ro;
    b->kmax[q] = std::max(1, d.lanczos_kmax);
    std::vector<int32_t> lrp(n + 1), lci(d.nnz);
    std::vector<double> lcv(d.nnz);
    if (d.nnz) {
      BH(hipMemcpy(lci.data(), d.col_idx, d.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
      BH(hipMemcpy(lcv.data(), d.val, d.nnz * sizeof(double), hipMemcpyDeviceToHost));
      if (d.ell_width > 0) {
        for (long i = 0; i <= n; ++i) lrp[i] = (int32_t)(i * d.ell_width);
      } else {
        BH(hipMemcpy(lrp.data(), d.row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
      }
    } else {
      std::fill(lrp.begin(), lrp.end(), 0);
    }
    if (d.validate && d.nnz && d.ell_width == 0) {
      std::string why;
      if (!check_csr(lrp, lci, n, d.nnz, why))
        return bail(fail(ALM_BM_ERR_INVALID_PATTERN, "instance " + std::to_string(q) + ": " + why));
    }
    if (d.diag) BH(hipMemcpy(dg.data() + ro, d.diag, n * sizeof(double), hipMemcpyDeviceToHost));
    BH(hipMemcpy(bb.data() + ro, d.b, n * sizeof(double), hipMemcpyDeviceToHost));
    double c2 = 0.0, b2 = 0.0;
    for (long i = 0; i < n; ++i) {
      for (int k = lrp[i]; k < lrp[i + 1]; ++k) {
        ci[ko] = lci[k] + (int32_t)ro;
        cv[ko] = lcv[k];
        c2 += lcv[k] * lcv[k];
        ++ko;
      }
      rp[ro + i + 1] = (int32_t)ko;
      c2 += dg[ro + i] * dg[ro + i];
      b2 += bb[ro + i] * bb[ro + i];
    }
    b->cnorm[q] = std::sqrt(c2);
    bnorm[q] = std::sqrt(b2);
    ro += n;
  }
  b->off[count] = ro;
  int32_t *drp, *dci;
  double *dcv, *ddg, *dbb;
  BK(balloc(b, (void**)&drp, (N + 1) * sizeof(int32_t)));
  BK(balloc(b, (void**)&dci, std::max<long>(1, ko) * sizeof(int32_t)));
  BK(balloc(b, (void**)&dcv, std::max<long>(1, ko) * sizeof(double)));
  BK(balloc(b, (void**)&ddg, N * sizeof(double)));
  BK(balloc(b, (void**)&dbb, N * sizeof(double)));
  BH(hipMemcpy(drp, rp.data(), (N + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  if (ko) BH(hipMemcpy(dci, ci.data(), ko * sizeof(int32_t), hipMemcpyHostToDevice));
  if (ko) BH(hipMemcpy(dcv, cv.data(), ko * sizeof(double), hipMemcpyHostToDevice));
  BH(hipMemcpy(ddg, dg.data(), N * sizeof(double), hipMemcpyHostToDevice));
  BH(hipMemcpy(dbb, bb.data(), N * sizeof(double), hipMemcpyHostToDevice));
  // ---- the super-problem handle
  alm_bm_problem_desc sd{};
  sd.n = N;
  sd.nnz = ko;
  sd.row_ptr = ko ? drp : nullptr;
  sd.col_idx = dci;
  sd.val = dcv;
  sd.ell_width = 0;
  sd.diag = ddg;
  sd.j_coef = 0.0;
  sd.cons_kind = ALM_BM_CONS_DIAG;
  sd.m = N;
  sd.b = dbb;
  sd.precision = prec;
  sd.r_max = rank_stride;
  sd.lanczos_kmax = kmax_all;
  sd.validate = 0;
  sd.rank_block_max = 0;
  sd.lbfgs_memory_max = lbm_all;  // rings of (sum n) x rank_stride elements per slot
  sd.hub_min_degree = -1;  // per-instance row widths: the hub sums (one stride r) do not apply
  BK(alm_bm_create(&sd, st, &b->p));
  alm_bm_problem* p = b->p;
  if (lbm_all > 0) BK(balloc(b, (void**)&p->lbs, (size_t)count * sizeof(LbfgsState)));
  // ---- block table: instance q gets ceil(n_q / rows_per_block) blocks
  const long rpb = std::max<long>(256, (N + 8191) / 8192);
  std::vector<int32_t> binst, iblo(count), ibhi(count);
  std::vector<int64_t> blo, bhi;
  for (int q = 0; q < count; ++q) {
    const long n = b->off[q + 1] - b->off[q];
    const long nbq = std::max<long>(1, (n + rpb - 1) / rpb);
    iblo[q] = (int32_t)binst.size();
    for (long k = 0; k < nbq; ++k) {
      binst.push_back(q);
      blo.push_back(b->off[q] + n * k / nbq);
      bhi.push_back(b->off[q] + n * (k + 1) / nbq);
    }
    ibhi[q] = (int32_t)binst.size();
  }
  const int nb = (int)binst.size();
  int32_t *dbinst, *diblo, *dibhi;
  int64_t *dblo, *dbhi;
  BK(balloc(b, (void**)&dbinst, nb * sizeof(int32_t)));
  BK(balloc(b, (void**)&dblo, nb * sizeof(int64_t)));
  BK(balloc(b, (void**)&dbhi, nb * sizeof(int64_t)));
  BK(balloc(b, (void**)&diblo, count * sizeof(int32_t)));
  BK(balloc(b, (void**)&dibhi, count * sizeof(int32_t)));
  BH(hipMemcpy(dbinst, binst.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice));
  BH(hipMemcpy(dblo, blo.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice));
  BH(hipMemcpy(dbhi, bhi.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice));
  BH(hipMemcpy(diblo, iblo.data(), count * sizeof(int32_t), hipMemcpyHostToDevice));
  BH(hipMemcpy(dibhi, ibhi.data(), count * sizeof(int32_t), hipMemcpyHostToDevice));
  p->tab = BlockTab{dbinst, dblo, dbhi, diblo, dibhi};
  p->count = count;
  p->nblk = nb;
  b->h_iblo = iblo;
  b->h_ibhi = ibhi;
  b->h_lo = blo;
  b->h_hi = bhi;
  for (int c = 0; c < alm_bm_batch::kNC; ++c) {
    BK(balloc(b, (void**)&b->c_inst[c], nb * sizeof(int32_t)));
    BK(balloc(b, (void**)&b->c_lo[c], nb * sizeof(int64_t)));
    BK(balloc(b, (void**)&b->c_hi[c], nb * sizeof(int64_t)));
    BK(balloc(b, (void**)&b->c_gid[c], nb * sizeof(int32_t)));
  }
  BK(balloc(b, (void**)&b->l_inst, nb * sizeof(int32_t)));
  BK(balloc(b, (void**)&b->l_lo, nb * sizeof(int64_t)));
  BK(balloc(b, (void**)&b->l_hi, nb * sizeof(int64_t)));
  BK(balloc(b, (void**)&b->l_gid, nb * sizeof(int32_t)));
  BK(balloc(b, (void**)&b->lm_dev, count * sizeof(int32_t)));
  BK(balloc(b, (void**)&b->xbase_dev, count * sizeof(int64_t)));
  BK(balloc(b, (void**)&b->ob_dev, count * sizeof(int64_t)));
  BK(balloc(b, (void**)&b->os_dev, count * sizeof(int32_t)));
  BK(balloc(b, (void**)&b->nbase_dev, count * sizeof(int64_t)));
  BK(balloc(b, (void**)&b->ns_dev, count * sizeof(int32_t)));
  BK(balloc(b, (void**)&b->nc_dev, count * sizeof(int32_t)));
  // ---- per-instance workspace sized for the table and the instance count
  const int kp = p->kmax + 1;
  BK(balloc(b, (void**)&p->part, (size_t)nb * (NUM_P + kMaxR) * sizeof(double)));
  BK(balloc(b, (void**)&p->part_c2, (size_t)nb * sizeof(double)));
  BK(balloc(b, (void**)&p->part_vec, (size_t)nb * 2 * sizeof(double)));
  BK(balloc(b, (void**)&p->sc_api, (size_t)count * sizeof(DevScalars)));
  BK(balloc(b, (void**)&p->sc_solve, (size_t)count * sizeof(DevScalars)));
  BH(hipMemset(p->sc_api, 0, (size_t)count * sizeof(DevScalars)));
  BH(hipMemset(p->sc_solve, 0, (size_t)count * sizeof(DevScalars)));
  p->lnb = nb;
  BK(balloc(b, (void**)&p->lpart, (size_t)nb * kp * sizeof(double)));
  BK(balloc(b, (void**)&p->lpart2, (size_t)nb * sizeof(double)));
  BK(balloc(b, (void**)&p->lh1, (size_t)count * kp * sizeof(double)));
  BK(balloc(b, (void**)&p->lh2, (size_t)count * kp * sizeof(double)));
  BK(balloc(b, (void**)&p->lalpha, (size_t)count * kp * sizeof(double)));
  BK(balloc(b, (void**)&p->lbeta, (size_t)count * kp * sizeof(double)));
  BK(balloc(b, (void**)&p->ls, (size_t)count * kp * sizeof(double)));
  BK(balloc(b, (void**)&p->lscal, (size_t)count * 4 * sizeof(double)));
  BK(balloc(b, (void**)&b->bnorm_dev, count * sizeof(double)));
  BK(balloc(b, (void**)&b->flags_dev, 2 * count * sizeof(int32_t)));
  BK(balloc(b, (void**)&b->tols_dev, count * sizeof(double)));
  BK(balloc(b, (void**)&b->active_dev, count * sizeof(int32_t)));
  BK(balloc(b, (void**)&b->col_dev, count * sizeof(int32_t)));
  BK(balloc(b, (void**)&b->scale_dev, count * sizeof(double)));
  BK(balloc(b, (void**)&b->thetas_dev, count * sizeof(double)));
  BH(hipMemcpy(b->bnorm_dev, bnorm.data(), count * sizeof(double), hipMemcpyHostToDevice));
  BH(hipDeviceSynchronize());
  *out = b;
  return ALM_BM_OK;
#undef BK
#undef BH
}

namespace {

struct BatchLanczos {
  std::vector<double> theta, resid;
  std::vector<int> m;
};

}  // namespace

// Launch order of a table's nb entries over the chip's eight XCDs.  The
// dispatcher hands workgroup i to XCD i mod 8, so launch position 8j + x gets
// entry j of XCD x's contiguous share of the table: each XCD walks one
// contiguous stretch of rows, a few instances at a time, and the vector
// entries those instances gather stay in its own L2 instead of being fetched
// by all eight.  Used for the Lanczos matvec (8-byte gathers: 1.7x faster on
// the uneven batch); the factor products keep the round-robin order, where
// the rows gathered do not fit one L2 either way and the contiguous shares
// (row-balanced, not nonzero-balanced) left the XCDs unevenly loaded.
static void xcd_order(std::vector<int32_t>& inst, std::vector<int64_t>& lo, std::vector<int64_t>& hi,
                      std::vector<int32_t>& gid) {
  constexpr int X = 8;
  const int nb = (int)inst.size();
  if (nb < 2 * X) return;
  int start[X + 1];
  start[0] = 0;
  for (int x = 0; x < X; ++x) start[x + 1] = start[x] + nb / X + (x < nb % X ? 1 : 0);
  std::vector<int32_t> i2(nb), g2(nb);
  std::vector<int64_t> l2(nb), h2(nb);
  for (int pos = 0; pos < nb; ++pos) {
    const int e = start[pos % X] + pos / X;
    i2[pos] = inst[e];
    l2[pos] = lo[e];
    h2[pos] = hi[e];
    g2[pos] = gid[e];
  }
  inst.swap(i2);
  lo.swap(l2);
  hi.swap(h2);
  gid.swap(g2);
}

// Launch table of the blocks of the instances with sel[q] != 0 (the Lanczos
// table); returns its block count.  Each block keeps its slot in the full
// table, so the per-instance reductions do not depend on the selection.
static alm_bm_status batch_lanczos_table(alm_bm_batch* b, const std::vector<char>& sel, int& nb, hipStream_t st) {
  b->hl_inst.clear();
  b->hl_lo.clear();
  b->hl_hi.clear();
  b->hl_gid.clear();
  for (int q = 0; q < b->count; ++q) {
    if (!sel[q]) continue;
    for (int blk = b->h_iblo[q]; blk < b->h_ibhi[q]; ++blk) {
      b->hl_inst.push_back(q);
      b->hl_lo.push_back(b->h_lo[blk]);
      b->hl_hi.push_back(b->h_hi[blk]);
      b->hl_gid.push_back(blk);
    }
  }
  xcd_order(b->hl_inst, b->hl_lo, b->hl_hi, b->hl_gid);
  nb = (int)b->hl_inst.size();
  if (nb == 0) return ALM_BM_OK;
  HIPCHK(hipMemcpyAsync(b->l_inst, b->hl_inst.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->l_lo, b->hl_lo.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->l_hi, b->hl_hi.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->l_gid, b->hl_gid.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));  // the table's host side is rebuilt by the next call
  return ALM_BM_OK;
}

// One Lanczos pass on Z(y) for the instances with run[q] != 0, in lockstep.
// Every 8 steps the host checks each running instance's Ritz residual; an
// instance that meets tol[q] (or exhausts its basis) leaves the launch table,
// so later steps cost only the instances still running.  Results of the
// other instances in `out` are left as they are.
// Start of a pass: 0 a random vector, 1 the Ritz vector in v (a restart),
// 2 the Ritz vector of the previous outer iteration in v plus a 10 % random
// share (a warm start).
static alm_bm_status batch_lanczos_pass(alm_bm_batch* b, const double* y, int kmax, const std::vector<double>& tol,
                                        uint64_t seed, int start, double* v, BatchLanczos& out, hipStream_t st,
                                        const std::vector<int32_t>& run) {
  alm_bm_problem* p = b->p;
  const int count = b->count;
  const long n = p->d.n, ldq = n;
  const int kp = p->kmax + 1;
  kmax = std::min(kmax, p->kmax);
  std::vector<char> live(count), done(count, 1);
  int ndone = count;
  for (int q = 0; q < count; ++q) {
    live[q] = run[q] != 0;
    if (live[q]) {
      done[q] = 0;
      --ndone;
      out.theta[q] = 0.0;
      out.resid[q] = 0.0;
      out.m[q] = 0;
    }
  }
  if (ndone == count) return ALM_BM_OK;
  int nb = 0;
  STCHK(batch_lanczos_table(b, live, nb, st));
  const BlockTab ltab{b->l_inst, b->l_lo, b->l_hi, p->tab.iblo, p->tab.ibhi, b->l_gid, nullptr};
  VecBatch vb{ltab, count, kp, kp};
  if (start == 1) {
    launch_resid(n, v, v, 0.0, nullptr, p->lpart2, nb, st, vb);
    launch_fin_sum(p->lpart2, nb, p->lscal, 1, st, vb, 4);
    launch_scale(n, v, p->lscal, p->Q, p->lpart2, nb, nullptr, st, vb, 4);
  } else {
    launch_rand(n, seed, p->lw, p->lpart2, nb, st, vb);
    launch_fin_sum(p->lpart2, nb, p->lscal, 1, st, vb, 4);
    if (start == 2) {
      launch_mix(n, 0.1, v, p->lw, p->lscal, 4, p->lpart2, nb, st, vb);
      launch_fin_sum(p->lpart2, nb, p->lscal, 1, st, vb, 4);
    }
    launch_scale(n, p->lw, p->lscal, p->Q, p->lpart2, nb, nullptr, st, vb, 4);
  }
  std::vector<double> ha((size_t)count * kp), hb((size_t)count * kp);
  std::vector<std::vector<double>> z(count);
  for (int j = 0; j < kmax; ++j) {
    const double* qj = p->Q + (long)j * ldq;
    launch_slack_mv_tab(p->C64, y, qj, p->lw, ltab, nb, st);
    launch_dots(n, j + 1, p->Q, ldq, p->lw, p->lpart, kp, nb, p->lh1, st, vb);
    launch_sub(n, j + 1, p->Q, ldq, p->lh1, p->lw, p->lpart2, nb, st, vb);
    launch_dots(n, j + 1, p->Q, ldq, p->lw, p->lpart, kp, nb, p->lh2, st, vb);
    launch_sub(n, j + 1, p->Q, ldq, p->lh2, p->lw, p->lpart2, nb, st, vb);
    launch_fin_ab(p->lpart2, nb, p->lh1, p->lh2, j, p->lalpha, p->lbeta, st, vb);
    launch_scale(n, p->lw, p->lbeta + j, p->Q + (long)(j + 1) * ldq, p->lpart2, nb, nullptr, st, vb, kp);
    const bool last = (j + 1 == kmax);
    if (((j + 1) % 8) == 0 || last) {
      HIPCHK(hipMemcpyAsync(ha.data(), p->lalpha, ha.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hb.data(), p->lbeta, hb.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      bool dropped = false;
      for (int q = 0; q < count; ++q) {
        if (done[q]) continue;
        std::vector<double> a(ha.begin() + (long)q * kp, ha.begin() + (long)q * kp + j + 1);
        std::vector<double> bt(hb.begin() + (long)q * kp, hb.begin() + (long)q * kp + j + 1);
        for (int i = 0; i <= j; ++i)
          if (!std::isfinite(a[i]) || !std::isfinite(bt[i])) return fail(ALM_BM_ERR_NUMERIC, "batch lanczos: NaN/Inf");
        double anorm = 0.0;
        for (int i = 0; i <= j; ++i) anorm = std::max(anorm, std::fabs(a[i]) + std::fabs(bt[i]));
        int mm = j + 1;
        bool breakdown = false;
        for (int i = 0; i <= j; ++i)
          if (bt[i] <= 1e-13 * std::max(anorm, 1e-300)) {
            mm = i + 1;
            breakdown = true;
            break;
          }
        const double th = tri_min_eig(a, bt, mm);
        tri_eigvec(a, bt, mm, th, z[q]);
        out.theta[q] = th;
        out.m[q] = mm;
        const double est = breakdown ? 0.0 : std::fabs(bt[mm - 1] * z[q][mm - 1]);
        if (breakdown || est <= tol[q] || mm >= b->kmax[q] || mm >= (int)(b->off[q + 1] - b->off[q])) {
          done[q] = 1;
          ++ndone;
          dropped = true;
        }
      }
      if (ndone == count || last) break;
      if (dropped) {
        for (int q = 0; q < count; ++q) live[q] = !done[q];
        STCHK(batch_lanczos_table(b, live, nb, st));
      }
    }
  }
  // Ritz vectors of the instances of this pass, each from its own basis size
  for (int q = 0; q < count; ++q) live[q] = run[q] != 0;
  STCHK(batch_lanczos_table(b, live, nb, st));
  int mmax = 1;
  std::vector<double> s((size_t)count * kp, 0.0);
  std::vector<int32_t> mq(count, 0);
  for (int q = 0; q < count; ++q) {
    if (!live[q]) continue;
    for (int i = 0; i < out.m[q]; ++i) s[(size_t)q * kp + i] = z[q][i];
    mq[q] = out.m[q];
    mmax = std::max(mmax, out.m[q]);
  }
  HIPCHK(hipMemcpyAsync(p->ls, s.data(), s.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->lm_dev, mq.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->thetas_dev, out.theta.data(), count * sizeof(double), hipMemcpyHostToDevice, st));
  launch_combine(n, mmax, p->Q, ldq, p->ls, v, p->lpart2, nb, st, vb, b->lm_dev);
  launch_fin_sum(p->lpart2, nb, p->lscal + 1, 1, st, vb, 4);
  launch_scale(n, v, p->lscal + 1, v, p->lpart2, nb, nullptr, st, vb, 4);
  launch_slack_mv_tab(p->C64, y, v, p->lw, ltab, nb, st);
  launch_resid(n, p->lw, v, 0.0, b->thetas_dev, p->lpart2, nb, st, vb);
  launch_fin_sum(p->lpart2, nb, p->lscal + 2, 1, st, vb, 4);
  std::vector<double> sc4((size_t)count * 4);
  HIPCHK(hipMemcpyAsync(sc4.data(), p->lscal, sc4.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  for (int q = 0; q < count; ++q)
    if (live[q]) out.resid[q] = sc4[(size_t)q * 4 + 2];
  return ALM_BM_OK;
}

// Lanczos for the instances with sel[q] != 0: a pass, then up to `restarts`
// passes from the Ritz vector for the instances whose Ritz residual still
// exceeds tol[q] (the others keep their results).  Entries of unselected
// instances are zero.
static alm_bm_status batch_lanczos(alm_bm_batch* b, const double* y, int kmax, const std::vector<double>& tol,
                                   uint64_t seed, double* v, BatchLanczos& out, hipStream_t st,
                                   const std::vector<int32_t>& sel, int restarts = 3, bool warm = false) {
  const int count = b->count;
  out.theta.assign(count, 0.0);
  out.resid.assign(count, 0.0);
  out.m.assign(count, 0);
  std::vector<int32_t> run(sel);
  for (int rs = 0; rs <= restarts; ++rs) {
    STCHK(batch_lanczos_pass(b, y, kmax, tol, seed, rs > 0 ? 1 : (warm ? 2 : 0), v, out, st, run));
    bool again = false;
    for (int q = 0; q < count; ++q) {
      run[q] = run[q] && out.resid[q] > tol[q];
      again = again || run[q];
    }
    if (!again) break;
  }
  return ALM_BM_OK;
}

// Row offset base of instance q stored at width w inside its region.
static int64_t batch_xbase(const alm_bm_batch* b, int q, int w) { return b->off[q] * (int64_t)(b->rs - w); }

// Re-lay every instance's factor out from (ob, os) to (nb, ns), keeping its
// first nc_q columns and zeroing the rest, through the handle's scratch.
template <typename T>
static alm_bm_status batch_restride(alm_bm_batch* b, T* R, const std::vector<int64_t>& ob,
                                    const std::vector<int32_t>& os, const std::vector<int64_t>& nbv,
                                    const std::vector<int32_t>& ns, const int32_t* nc, hipStream_t st) {
  alm_bm_problem* p = b->p;
  const int count = b->count;
  HIPCHK(hipMemcpyAsync(b->ob_dev, ob.data(), count * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->os_dev, os.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->nbase_dev, nbv.data(), count * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->ns_dev, ns.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(b->nc_dev, nc, count * sizeof(int32_t), hipMemcpyHostToDevice, st));
  T* Rt = static_cast<T*>(p->Rtmp);
  launch_restride_batch<T>(p->tab, p->nblk, R, Rt, b->ob_dev, b->os_dev, b->nbase_dev, b->ns_dev, b->nc_dev, st);
  HIPCHK(hipMemcpyAsync(R, Rt, (size_t)p->d.n * b->rs * sizeof(T), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));  // the host argument vectors may go out of scope
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

// Launch tables of the active instances, one per distinct width, and the
// per-instance row bases of the current widths.
static alm_bm_status batch_classes(alm_bm_batch* b, const std::vector<int>& w, const std::vector<int32_t>& active,
                                   hipStream_t st) {
  const int count = b->count;
  std::vector<int> widths;
  for (int q = 0; q < count; ++q)
    if (active[q] && std::find(widths.begin(), widths.end(), w[q]) == widths.end()) widths.push_back(w[q]);
  if ((int)widths.size() > alm_bm_batch::kNC) return fail(ALM_BM_ERR_UNSUPPORTED, "batch: too many width classes");
  std::sort(widths.begin(), widths.end());
  std::vector<std::vector<int32_t>> ci(widths.size()), cg(widths.size());
  std::vector<std::vector<int64_t>> cl(widths.size()), ch(widths.size());
  for (int q = 0; q < count; ++q) {
    if (!active[q]) continue;
    const int c = (int)(std::find(widths.begin(), widths.end(), w[q]) - widths.begin());
    for (int blk = b->h_iblo[q]; blk < b->h_ibhi[q]; ++blk) {
      ci[c].push_back(q);
      cl[c].push_back(b->h_lo[blk]);
      ch[c].push_back(b->h_hi[blk]);
      cg[c].push_back(blk);
    }
  }
  b->nclass = (int)widths.size();
  for (int c = 0; c < b->nclass; ++c) {
    const size_t k = ci[c].size();
    b->c_nb[c] = (int)k;
    b->c_w[c] = widths[c];
    const auto it = b->wvar.find(widths[c]);
    b->c_var[c] = it == b->wvar.end() ? 0 : it->second;
    HIPCHK(hipMemcpyAsync(b->c_inst[c], ci[c].data(), k * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->c_lo[c], cl[c].data(), k * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->c_hi[c], ch[c].data(), k * sizeof(int64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->c_gid[c], cg[c].data(), k * sizeof(int32_t), hipMemcpyHostToDevice, st));
  }
  std::vector<int64_t> xb(count);
  for (int q = 0; q < count; ++q) xb[q] = batch_xbase(b, q, w[q]);
  HIPCHK(hipMemcpyAsync(b->xbase_dev, xb.data(), count * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return ALM_BM_OK;
}

static BlockTab batch_class_tab(const alm_bm_batch* b, int c) {
  const BlockTab& f = b->p->tab;
  return BlockTab{b->c_inst[c], b->c_lo[c], b->c_hi[c], f.iblo, f.ibhi, b->c_gid[c], b->xbase_dev};
}

// One inner step of every running instance: each row kernel once per width.
template <typename T>
static void batch_enqueue_step(alm_bm_batch* b, T* R, const double* y, double sigma, T* G, int refresh,
                               hipStream_t st) {
  using V = typename Acc<T>::type;
  alm_bm_problem* p = b->p;
  const auto& d = p->d;
  DevScalars* sc = p->sc_solve;
  V* Q = static_cast<V*>(p->Qbuf);
  using S = RingT<T>;
  const LbfgsRing<S> lb = lbfgs_ring<S>(p);  // empty: gradient descent
  for (int c = 0; c < b->nclass; ++c)
    launch_upd_eval_diag<T>(d.n, b->c_w[c], b->c_var[c], R, G, Q, y, d.b, sigma, p->Av, p->part, sc, refresh,
                            batch_class_tab(b, c), b->c_nb[c], st, lb);
  for (int c = 0; c < b->nclass; ++c)
    launch_objgrad_diag<T>(cost_of<T>(p), b->c_w[c], b->c_var[c], R, y, d.b, sigma, G, p->Av, p->part, sc, refresh,
                           batch_class_tab(b, c), b->c_nb[c], st, lb);
  launch_fin_objgrad(p->part, p->nblk, sc, sigma, 1, nullptr, st, p->tab, p->count);
  if (lb.s) {
    // L-BFGS per instance: states, ring regions and partial slots follow the
    // block table, so one launch per width class covers every instance
    for (int c = 0; c < b->nclass; ++c)
      launch_lbfgs_dots<T>(d.n, b->c_w[c], G, lb, p->part, b->c_nb[c], sc, st, batch_class_tab(b, c));
    launch_fin_lbfgs(p->part, p->nblk, sc, lb.s, st, p->tab, p->count);
    for (int c = 0; c < b->nclass; ++c)
      launch_lbfgs_combine<T>(d.n, b->c_w[c], b->c_var[c], R, G, y, d.b, sigma, p->Av, lb, p->part, sc,
                              b->c_nb[c], st, batch_class_tab(b, c));
    launch_fin_lsdir(p->part, p->nblk, sc, lb.s, st, p->tab, p->count);
    for (int c = 0; c < b->nclass; ++c)
      launch_quadq_diag<S>(cost_of<S>(p), b->c_w[c], b->c_var[c], lb.e, Q, p->part_c2, sc, batch_class_tab(b, c),
                           b->c_nb[c], st, lb);
  } else {
    for (int c = 0; c < b->nclass; ++c)
      launch_quadq_diag<T>(cost_of<T>(p), b->c_w[c], b->c_var[c], G, Q, p->part_c2, sc, batch_class_tab(b, c),
                           b->c_nb[c], st);
  }
  launch_fin_step(p->part_c2, p->nblk, 1, sc, sigma, 0.0, 1, nullptr, nullptr, st, p->tab, p->count);
}

// Objective pass (API mode, into sc_api) over the active instances.
template <typename T>
static void batch_enqueue_objgrad(alm_bm_batch* b, const T* R, const double* y, double sigma, hipStream_t st) {
  alm_bm_problem* p = b->p;
  for (int c = 0; c < b->nclass; ++c)
    launch_objgrad_diag<T>(cost_of<T>(p), b->c_w[c], b->c_var[c], R, y, p->d.b, sigma, nullptr, p->Av, p->part,
                           p->sc_api, 0, batch_class_tab(b, c), b->c_nb[c], st);
  launch_fin_objgrad(p->part, p->nblk, p->sc_api, sigma, 0, nullptr, st, p->tab, p->count);
}

template <typename T>
static alm_bm_status batch_solve_impl(alm_bm_batch* b, const alm_bm_options& o, T* R, int32_t* r, double* y,
                                      alm_bm_result* results, int32_t* status, hipStream_t st) {
  alm_bm_problem* p = b->p;
  const int count = b->count;
  const long N = p->d.n;
  const double sigma = o.sigma;
  const double t0 = now_s();
  const int refresh = o.refresh_every > 0 ? o.refresh_every
                                          : default_refresh(sizeof(T) == 8 ? ALM_BM_F64
                                                                           : (sizeof(T) == 4 ? ALM_BM_F32 : ALM_BM_BF16));
  const int U = std::max(1, o.graph_unroll);
  const int kmax = o.lanczos_kmax > 0 ? std::min(o.lanczos_kmax, p->kmax) : p->kmax;
  std::vector<double> tolv(count), pinf_prev(count, INFINITY), tol_prev(count, INFINITY), tau(count), ltol(count);
  std::vector<int> rcap(count);
  std::vector<int32_t> active(count, 1), st_q(count, ALM_BM_NOT_CONVERGED);
  std::vector<alm_bm_result> res(count);
  for (int q = 0; q < count; ++q) {
    const long nq = b->off[q + 1] - b->off[q];
    rcap[q] = std::min(b->rs, bp_rank_cap(nq));
    if (o.r_cap > 0) rcap[q] = std::min(rcap[q], o.r_cap);
    tau[q] = o.tau_rank > 0.0 ? o.tau_rank : o.eps_kkt * (1.0 + b->cnorm[q]);
    ltol[q] = o.lanczos_tol_rel * o.eps_kkt * (1.0 + b->cnorm[q]);
    res[q] = alm_bm_result{};
    res[q].promoted_at_outer = -1;
    if (r[q] < 1 || r[q] > b->rs) return fail(ALM_BM_ERR_INVALID_ARG, "batch_solve: r[q] must be in 1..rank_stride");
  }
  T* G = static_cast<T*>(p->G);
  // per-instance widths: pack from the caller's layout (row i at i * rs)
  std::vector<int> w(count);
  std::vector<int64_t> xb(count), zero64(count, 0);
  std::vector<int32_t> rsv(count, b->rs), wv(count);
  for (int q = 0; q < count; ++q) {
    w[q] = pad_width(r[q], b->rs);
    wv[q] = w[q];
    xb[q] = batch_xbase(b, q, w[q]);
  }
  STCHK(batch_restride<T>(b, R, zero64, rsv, xb, wv, r, st));
  GraphCache gc;
  // The launch tables and the captured step depend only on the widths and the
  // running set: both are rebuilt when either changed since they were made.
  std::vector<int> tab_w, gr_w;
  std::vector<int32_t> tab_active, gr_active;
  int captures = 0;
  std::vector<int32_t> fl(2 * count);
  int nactive = count;
  for (int k = 0; k < o.max_outer && nactive > 0; ++k) {
    for (int q = 0; q < count; ++q) {
      if (!active[q]) continue;
      tolv[q] = std::max(o.eps_kkt / 10.0, std::min(o.inner_tol_scale, std::min(pinf_prev[q], o.inner_tol_decay * tol_prev[q])));
      tol_prev[q] = tolv[q];
    }
    // launch tables of this outer iteration's running instances, and the graph
    const double ti = now_s();
    if (w != tab_w || active != tab_active) {
      STCHK(batch_classes(b, w, active, st));
      tab_w = w;
      tab_active = active;
    }
    if (!gc.exec || w != gr_w || active != gr_active) {
      gc.reset();
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      for (int u = 0; u < U; ++u) batch_enqueue_step<T>(b, R, y, sigma, G, refresh, st);
      HIPCHK(hipStreamEndCapture(st, &gc.graph));
      HIPCHK(hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0));
      gr_w = w;
      gr_active = active;
      ++captures;
    }
    HIPCHK(hipMemcpyAsync(b->tols_dev, tolv.data(), count * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->active_dev, active.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, st));
    launch_inner_reset_batch(p->sc_solve, count, b->tols_dev, b->active_dev, o.max_inner, (int)o.step_rule,
                             o.eta_fixed, st);
    if (p->lb_m > 0) launch_lbfgs_reset(p->lbs, p->lb_m, st, count);  // empty memories
    int launched = 0;
    while (true) {
      HIPCHK(hipGraphLaunch(gc.exec, st));
      launched += U;
      launch_gather_flags(p->sc_solve, count, b->flags_dev, st);
      HIPCHK(hipMemcpyAsync(fl.data(), b->flags_dev, 2 * count * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      bool all = true;
      for (int q = 0; q < count; ++q)
        if (fl[2 * q] == 0) all = false;
      if (all) break;
      if (launched > o.max_inner + 2 * U + 2) return fail(ALM_BM_ERR_HIP, "batch inner loop did not reach its stop flags");
    }
    for (int q = 0; q < count; ++q)
      if (active[q]) res[q].inner_total += fl[2 * q + 1];
    const double tinner = now_s() - ti;
    // w = y - sigma (A(RR^T) - b) for every instance
    launch_dual_batch(N, p->Av, p->d.b, y, p->ybuf, sigma, p->part_vec, p->sc_solve, b->bnorm_dev, p->tab, p->nblk,
                      count, st);
    BatchLanczos L;
    const double tl = now_s();
    // from the second outer iteration on, each instance's pass starts from its
    // previous Ritz vector (plus a random share): the dual moved only a little
    STCHK(batch_lanczos(b, p->ybuf, kmax, ltol, o.seed * 1000003ull + (uint64_t)k, p->lv, L, st, active,
                        o.lanczos_restarts, k > 0));
    const double tlan = now_s() - tl;
    // KKT per instance at the point as it stands (R, the updated dual):
    // <C, RR^T> and pinf at R, b^T y at y; the final values unless a rank step
    // follows
    std::vector<DevScalars> hs(count);
    auto batch_kkt = [&](const double* yv) -> alm_bm_status {
      batch_enqueue_objgrad<T>(b, R, yv, 0.0, st);
      launch_dual_batch(N, p->Av, p->d.b, yv, nullptr, 0.0, p->part_vec, p->sc_api, b->bnorm_dev, p->tab, p->nblk,
                        count, st);
      HIPCHK(hipMemcpyAsync(hs.data(), p->sc_api, count * sizeof(DevScalars), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipGetLastError());
      return ALM_BM_OK;
    };
    STCHK(batch_kkt(p->ybuf));
    // rank expansion decisions (the rank test of Alg. 1, plus the blocked
    // certificate case of the single solve)
    std::vector<int32_t> col(count, 0);
    std::vector<double> scale(count, -1.0);
    std::vector<char> expanded(count, 0);
    bool any = false;
    if (o.rank_policy == ALM_BM_RANK_ADAPT) {
      VecBatch vb{p->tab, count, p->kmax + 1, p->kmax + 1};
      launch_quartic_norm(N, 0, p->adj, p->lv, p->lpart2, p->nblk, st, vb);
      launch_fin_sum(p->lpart2, p->nblk, p->lscal + 3, 0, st, vb, 4);
      std::vector<double> sc4((size_t)count * 4);
      HIPCHK(hipMemcpyAsync(sc4.data(), p->lscal, sc4.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (int q = 0; q < count; ++q) {
        if (!active[q]) continue;
        const bool gate = (fl[2 * q] == 1) || !o.expand_needs_inner;
        const double q4 = sc4[(size_t)q * 4 + 3];
        KktVals k0{};
        const double rq0 = slack_rq(hs[q].tot[P_C0], hs[q].dobj, hs[q].tot[P_YBMA], hs[q].tot[P_RR]);
        kkt_terms(hs[q].tot[P_C0], hs[q].dobj, hs[q].pinf, L.theta[q], rq0, b->cnorm[q], k0);
        const double dtol = o.eps_kkt * (1.0 + b->cnorm[q]);
        const bool blocked = k0.kkt <= o.eps_kkt && L.resid[q] < dtol && L.resid[q] - L.theta[q] > dtol;
        const double tau_q = blocked ? 0.0 : tau[q];
        if (gate && L.theta[q] < -tau_q && r[q] < rcap[q] && q4 > 0.0) {
          col[q] = r[q];
          scale[q] = std::sqrt(std::max(0.0, -L.theta[q] / (sigma * q4)));
          expanded[q] = 1;
          res[q].expansions += 1;
          any = true;
        }
      }
      if (any) {
        // widen the instances whose new column does not fit their width
        std::vector<int> w2(w);
        bool widen = false;
        for (int q = 0; q < count; ++q)
          if (expanded[q] && r[q] + 1 > w[q]) {
            w2[q] = pad_width(r[q] + 1, b->rs);
            widen = true;
          }
        if (widen) {
          std::vector<int64_t> ob(count), nbv(count);
          std::vector<int32_t> os(count), ns(count);
          for (int q = 0; q < count; ++q) {
            ob[q] = batch_xbase(b, q, w[q]);
            os[q] = w[q];
            nbv[q] = batch_xbase(b, q, w2[q]);
            ns[q] = w2[q];
          }
          STCHK(batch_restride<T>(b, R, ob, os, nbv, ns, r, st));
          w = w2;
          STCHK(batch_classes(b, w, active, st));
          tab_w = w;
          tab_active = active;
        }
        for (int q = 0; q < count; ++q)
          if (expanded[q]) r[q] += 1;
        HIPCHK(hipMemcpyAsync(b->col_dev, col.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(b->scale_dev, scale.data(), count * sizeof(double), hipMemcpyHostToDevice, st));
        for (int c = 0; c < b->nclass; ++c)
          launch_fill_column<T>(N, b->c_w[c], R, p->lv, b->col_dev, b->scale_dev, batch_class_tab(b, c), b->c_nb[c],
                                st);
        batch_enqueue_objgrad<T>(b, R, y, sigma, st);
        launch_dual_batch(N, p->Av, p->d.b, y, p->ybuf, sigma, p->part_vec, p->sc_solve, b->bnorm_dev, p->tab,
                          p->nblk, count, st);
      }
    }
    launch_copy_active(N, p->ybuf, y, b->active_dev, p->tab, p->nblk, st);
    std::vector<double> lam(L.theta), lres(L.resid);
    double tlan2 = 0.0;
    if (any) {
      BatchLanczos L2;
      const double t2 = now_s();
      std::vector<int32_t> exp_sel(expanded.begin(), expanded.end());
      STCHK(batch_lanczos(b, y, kmax, ltol, o.seed * 1000003ull + (uint64_t)k + 7777777ull, p->lv, L2, st, exp_sel,
                          o.lanczos_restarts));
      tlan2 = now_s() - t2;
      for (int q = 0; q < count; ++q)
        if (expanded[q]) {
          lam[q] = L2.theta[q];
          lres[q] = L2.resid[q];
        }
    }
    if (any) STCHK(batch_kkt(y));  // after rank steps: the KKT at the new point
    for (int q = 0; q < count; ++q) {
      if (!active[q]) continue;
      KktVals kv{};
      const double rq = slack_rq(hs[q].tot[P_C0], hs[q].dobj, hs[q].tot[P_YBMA], hs[q].tot[P_RR]);
      kkt_terms(hs[q].tot[P_C0], hs[q].dobj, hs[q].pinf, lam[q], rq, b->cnorm[q], kv);
      if (!std::isfinite(kv.kkt))
        return fail(ALM_BM_ERR_NUMERIC, "batch_solve: non-finite KKT in instance " + std::to_string(q));
      res[q].outer = k + 1;
      res[q].rank = r[q];
      res[q].pobj = kv.pobj;
      res[q].dobj = kv.dobj;
      res[q].pinf = kv.pinf;
      res[q].dinf = kv.dinf;
      res[q].gap = kv.gap;
      res[q].kkt = kv.kkt;
      res[q].lam_min = std::min(lam[q], rq);
      res[q].lanczos_resid = lres[q];
      res[q].time_lanczos_s += (tlan + tlan2) / nactive;
      pinf_prev[q] = kv.pinf;
      if (kv.kkt <= o.eps_kkt && lanczos_certifies(lam[q], lres[q], ltol[q], rq, o.eps_kkt * (1.0 + b->cnorm[q]))) {
        active[q] = 0;
        st_q[q] = ALM_BM_OK;
        res[q].time_s = now_s() - t0;
        --nactive;
      }
    }
    if (o.verbose)
      std::fprintf(stderr,
                   "[almbm batch] k=%d active=%d t=%.2fs (inner %.3fs, %d graph launches, %d captures; "
                   "lanczos %.3fs)\n",
                   k, nactive, now_s() - t0, tinner, launched / U, captures, tlan + tlan2);
    if (o.time_limit_s > 0.0 && now_s() - t0 > o.time_limit_s) break;
  }
  // back to the caller's layout
  {
    std::vector<int64_t> ob(count);
    std::vector<int32_t> os(count);
    for (int q = 0; q < count; ++q) {
      ob[q] = batch_xbase(b, q, w[q]);
      os[q] = w[q];
    }
    STCHK(batch_restride<T>(b, R, ob, os, zero64, rsv, r, st));
  }
  for (int q = 0; q < count; ++q) {
    if (active[q]) res[q].time_s = now_s() - t0;
    if (results) results[q] = res[q];
    if (status) status[q] = st_q[q];
  }
  return nactive == 0 ? ALM_BM_OK : ALM_BM_NOT_CONVERGED;
}

// Tile choice per width: every width a batched solve can give an instance
// (pad_width of 1..rank_stride) is timed with all instances at that width,
// one objective/gradient pass over the whole block table per repetition and
// variant, on a zero factor in the handle's scratch (the gathers do not
// depend on the values).
template <typename T>
static alm_bm_status batch_autotune_impl(alm_bm_batch* b, int reps, hipStream_t st) {
  alm_bm_problem* p = b->p;
  const int count = b->count;
  const auto& d = p->d;
  std::vector<int> widths;
  for (int r = 1; r <= b->rs; ++r) {
    const int w = pad_width(r, b->rs);
    if (std::find(widths.begin(), widths.end(), w) == widths.end()) widths.push_back(w);
  }
  HIPCHK(hipMemsetAsync(p->Rtmp, 0, (size_t)d.n * b->rs * sizeof(T), st));
  HIPCHK(hipMemsetAsync(p->ybuf, 0, (size_t)d.m * sizeof(double), st));
  const T* R = static_cast<const T*>(p->Rtmp);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  std::vector<int32_t> all(count, 1);
  alm_bm_status s = ALM_BM_OK;
  for (int w : widths) {
    std::vector<int> wq(count, w);
    b->wvar.erase(w);
    s = batch_classes(b, wq, all, st);
    if (s != ALM_BM_OK) break;
    float best = INFINITY;
    int bv = 0;
    for (int v = 0; v <= 2; ++v) {
      auto run = [&]() {
        launch_objgrad_diag<T>(cost_of<T>(p), w, v, R, p->ybuf, d.b, 1.0, nullptr, p->Av, p->part, p->sc_api, 0,
                               batch_class_tab(b, 0), b->c_nb[0], st);
      };
      run();  // warm
      if (hipEventRecord(e0, st) != hipSuccess) s = fail(ALM_BM_ERR_HIP, "batch_autotune: event record");
      for (int k = 0; k < reps && s == ALM_BM_OK; ++k) run();
      if (s == ALM_BM_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
        s = fail(ALM_BM_ERR_HIP, "batch_autotune: event wait");
      float ms = 0.f;
      if (s == ALM_BM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        s = fail(ALM_BM_ERR_HIP, "batch_autotune: elapsed time");
      if (s != ALM_BM_OK) break;
      // another variant must beat the default by 3 %: differences inside the
      // timing noise would make the choice, and with it the rounding of the
      // row sums and the solve's trajectory, change from run to run
      if (v == 0 || ms < 0.97f * best) {
        best = ms;
        bv = v;
      }
    }
    if (s != ALM_BM_OK) break;
    b->wvar[w] = bv;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  STCHK(s);
  HIPCHK(hipGetLastError());
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_batch_autotune(alm_bm_batch* b, int32_t reps, int32_t* widths_out,
                                               int32_t* variants_out, int32_t* n_out, hipStream_t st_user) {
  if (!b) return fail(ALM_BM_ERR_INVALID_ARG, "batch_autotune: null handle");
  if (reps < 1) return fail(ALM_BM_ERR_INVALID_ARG, "batch_autotune: reps < 1");
  HIPCHK(hipStreamSynchronize(st_user));
  hipStream_t st = b->p->ss;
  STCHK(with_storage(b->p->d.precision, [&]<typename T>() { return batch_autotune_impl<T>(b, reps, st); }));
  HIPCHK(hipStreamSynchronize(st));
  int k = 0;
  for (const auto& [w, v] : b->wvar) {
    if (k < ALM_BM_BATCH_TUNE_MAX) {
      if (widths_out) widths_out[k] = w;
      if (variants_out) variants_out[k] = v;
    }
    ++k;
  }
  if (n_out) *n_out = std::min(k, ALM_BM_BATCH_TUNE_MAX);
  return ALM_BM_OK;
}

extern "C" alm_bm_status alm_bm_batch_solve(alm_bm_batch* b, const alm_bm_options* opts, void* R, int32_t* r,
                                            double* y, alm_bm_result* results, int32_t* status, hipStream_t st_user) {
  if (!b || !R || !r || !y) return fail(ALM_BM_ERR_INVALID_ARG, "batch_solve: null argument");
  alm_bm_options o;
  if (opts) o = *opts;
  else alm_bm_default_options(&o);
  if (!(o.sigma > 0.0) || !(o.eps_kkt > 0.0) || o.max_outer < 1 || o.max_inner < 1)
    return fail(ALM_BM_ERR_INVALID_ARG, "batch_solve: sigma, eps_kkt, max_outer and max_inner must be positive");
  if (o.sigma_growth != 1.0)
    return fail(ALM_BM_ERR_UNSUPPORTED, "batch_solve: the penalty schedule (sigma_growth) is for single solves");
  if (o.rank_block != 1) return fail(ALM_BM_ERR_UNSUPPORTED, "batch_solve: rank_block > 1 is for single solves");
  int lb_m = 0;
  if (o.inner_solver == ALM_BM_INNER_LBFGS) {
    if (o.lbfgs_memory < 1 || o.lbfgs_memory > b->p->d.lbfgs_memory_max)
      return fail(ALM_BM_ERR_INVALID_ARG, "batch_solve: lbfgs_memory must be in 1..the largest lbfgs_memory_max of "
                                          "the instances (" + std::to_string(b->p->d.lbfgs_memory_max) + ")");
    lb_m = o.lbfgs_memory;
  } else if (o.inner_solver != ALM_BM_INNER_GD) {
    return fail(ALM_BM_ERR_INVALID_ARG, "batch_solve: unknown inner_solver");
  }
  if (o.resume_outer != 0) return fail(ALM_BM_ERR_UNSUPPORTED, "batch_solve: resume is for single solves");
  HIPCHK(hipStreamSynchronize(st_user));
  hipStream_t st = b->p->ss;
  InnerScope inner_scope(b->p, lb_m);
  alm_bm_status s = with_storage(b->p->d.precision, [&]<typename T>() {
    return batch_solve_impl<T>(b, o, static_cast<T*>(R), r, y, results, status, st);
  });
  HIPCHK(hipStreamSynchronize(st));
  return s;
}
