// Kernel argument structures, device scalar block and launcher declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace almbm {

// Per-row partial sums produced by the objective/gradient pass.  Index names
// follow the quartic line search: a1 = A(RG^T + GR^T), a2 = A(GG^T), e = A(RR^T) - b.
enum PartialSlot {
  P_C0 = 0,    // <C, RR^T> (cost part; the -j J part is added at finalize)
  P_YBMA,      // <y, b - a>
  P_EE,        // ||e||^2
  P_GG,        // ||G||_F^2
  P_GP,        // <G, CR>
  P_YA1, P_YA2, P_EA1, P_EA2, P_A1A1, P_A1A2, P_A2A2,
  P_RR,        // ||R||_F^2
  P_RG,        // <R, G>      (edge family trace terms)
  P_C2,        // <G, CG>     (cost part)
  NUM_P
};

constexpr int kMaxR = 128;
constexpr int kMaxBlockQ = 8;  // block size of the block Krylov eigensolver

// Device-resident scalars of one handle.  Written by finalize kernels so that
// the inner loop needs no host round trip; the host reads them after syncs.
struct DevScalars {
  double tot[NUM_P];
  double f;               // objective at the current R
  double coeffs[5];       // quartic phi(t) coefficients
  double t;               // step chosen
  double tol;             // inner stop tolerance (host sets per outer iteration)
  double sigma;
  double eta_fixed;
  double pinf;
  double dobj;
  double res2;
  double w0;              // edge family: trace-row multiplier y0 - sigma (a0 - b0)
  double a0;              // edge family: trace_coef ||R||^2
  double qsum;            // sum of a Lanczos vector (for the -j J term)
  double colsum[kMaxR];   // edge family / J term: 1^T R
  double gcolsum[kMaxR];  // 1^T G
  int32_t flag;           // 0 running, 1 inner tolerance met, 2 max_inner reached
  int32_t iter;           // inner iterations taken
  int32_t max_inner;
  int32_t step_rule;      // 0 exact, 1 fixed
  int32_t numeric_error;  // set when a finalize sees NaN/Inf
  int32_t pad;
};

// ---- L-BFGS subproblem solver (limited-memory BFGS with the exact quartic
// line search; the solver of the SDPLR code that Sec. 2 names) ---------------
//
// The direction is E = H G with H the L-BFGS inverse-Hessian estimate from the
// last m pairs (s, y), s = R_new - R = -t E_old, y = G_new - G_old, and the
// step R <- R - t E takes the exact minimiser t of the quartic along -E.  The
// two-loop recursion runs on the coefficients of E in the basis {G, E_a, y_a}
// from inner products kept on the device (s_a^T y_b, y_a^T y_b, and the new
// gradient's products with every stored vector), so a step streams each
// stored vector twice (once for the inner products, once to form E) instead
// of 4m times.
constexpr int kMaxLbfgs = 8;
constexpr int kLbfgsSlots = kMaxLbfgs + 1;   // ring slots of E and of y
constexpr int kLbfgsDots = 5 * kLbfgsSlots;  // inner-product partial slots per block

struct LbfgsState {
  int32_t m;                       // pairs kept (1..kMaxLbfgs)
  int32_t cnt;                     // pairs held
  int32_t cur;                     // slot of the direction E_k (and of y_k)
  int32_t have;                    // a direction was taken (a pair candidate exists)
  int32_t ord[kMaxLbfgs];          // slots of the held pairs, oldest first
  int32_t resets;                  // memory clears (non-descent direction or zero step)
  int32_t accepted;                // pairs taken
  double tp[kLbfgsSlots];          // step taken along the direction in each slot (s = -t E)
  double ee;                       // ||E_k||^2
  double SY[kMaxLbfgs][kMaxLbfgs]; // s_a^T y_b (pairs in set order)
  double YY[kMaxLbfgs][kMaxLbfgs]; // y_a^T y_b
  double cg;                       // E_{k+1} = cg G + sum_a (ce[a] E_ord[a] + cy[a] y_ord[a])
  double ce[kMaxLbfgs], cy[kMaxLbfgs];
};

// Storage type of the rings: double for FP64 handles, bfloat16 otherwise.  The
// rings only shape the direction; the exact line search then runs along the
// direction as stored, so reduced ring precision never breaks descent (a
// direction that fails the descent test clears the memory).
template <typename T> struct RingOf { using type = bf16; };
template <> struct RingOf<double> { using type = double; };
template <typename T> using RingT = typename RingOf<T>::type;

// Device rings of one handle: slot s of E at e + s * stride, of y at y + s * stride.
template <typename T> struct LbfgsRing {
  LbfgsState* s = nullptr;
  T* e = nullptr;
  T* y = nullptr;
  long stride = 0;
};

// Sparse symmetric cost S (off-diagonal) + diagonal, in arithmetic type V.
template <typename V> struct Cost {
  long n;
  const int32_t* rp;   // CSR row pointers (nullptr for ELL)
  const int32_t* ci;
  const V* cv;
  int32_t ell;         // > 0: ELL width
  const V* dg;         // nullable
  // Hub rows (CSR, single instance): the nh rows with more than hthr stored
  // entries, in increasing order in hrow.  Before a row kernel multiplies C
  // with X, a block-per-hub kernel writes sum_k S_ik X_k of every hub into
  // hsum (row h of an nh x r array); the row kernel reads that sum instead of
  // walking the long row with one lane group.  hsum2 holds the second product
  // of a kernel that multiplies two operands.
  int32_t nh = 0;
  int32_t hthr = 0;
  const int32_t* hrow = nullptr;
  V* hsum = nullptr;
  V* hsum2 = nullptr;
};

// Position of hub row i in C.hrow (i must be a hub).
template <typename V>
__device__ __forceinline__ int hub_index(const Cost<V>& C, long i) {
  int lo = 0, hi = C.nh - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (C.hrow[mid] < i) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Edge family adjacency: symmetric pattern with edge ids, plus the upper
// (i < j) half in edge order (edge e sits at position e of the upper arrays).
struct EdgeAdj {
  const int32_t* rp;    // n+1, symmetric
  const int32_t* ci;    // 2E
  const int32_t* eid;   // 2E
  const int32_t* urp;   // n+1, upper half; urp[i]..urp[i+1] are edges with ei = i
  const int32_t* uci;   // E, = edge_j in edge order
  float avg_deg = 0.f;  // 2E / n: long rows (matrix completion) are split over several lane groups
};

// Batched mode: many instances concatenated block-diagonally.  Every block of
// a row kernel owns rows [lo, hi) of exactly one instance, so that per-block
// partial sums belong to one instance; instance q owns blocks [iblo, ibhi).
// A null table means a single instance with the default row chunking.
struct BlockTab {
  const int32_t* inst = nullptr;  // per block
  const int64_t* lo = nullptr;    // per block, first row
  const int64_t* hi = nullptr;    // per block, end row
  const int32_t* iblo = nullptr;  // per instance, first block
  const int32_t* ibhi = nullptr;  // per instance, end block
  // Optional, for launches over a subset of the blocks whose instances share
  // one row width r: the partial-sum slot of each launched block (its index
  // in the full table), and per instance the element offset xbase such that
  // row i of the factor starts at xbase + i * r.
  const int32_t* gid = nullptr;
  const int64_t* xbase = nullptr;
};

__device__ __forceinline__ long part_slot(const BlockTab& t) { return t.gid ? t.gid[blockIdx.x] : blockIdx.x; }
__device__ __forceinline__ long row_base(const BlockTab& t, int inst) { return t.xbase ? t.xbase[inst] : 0; }

struct Rows {
  long lo, hi;
  int inst;
};

__device__ __forceinline__ Rows rows_of(long n, const BlockTab& t) {
  if (!t.inst) {
    const RowChunk c = row_chunk(n);
    return {c.lo, c.hi, 0};
  }
  return {(long)t.lo[blockIdx.x], (long)t.hi[blockIdx.x], t.inst[blockIdx.x]};
}

// Lanczos vector kernels in batched mode: the table, the instance count and
// the per-instance strides of the projection coefficients (h), of the
// tridiagonal entries (alpha, beta) and of scalar outputs.
struct VecBatch {
  BlockTab tab{};
  int count = 1;
  int hstride = 0;
  int astride = 0;
};

// Block range of instance `q` for a finalize kernel (single mode: [0, nb)).
__device__ __forceinline__ void inst_blocks(const BlockTab& t, int q, int nb, int& b0, int& b1) {
  if (!t.iblo) {
    b0 = 0;
    b1 = nb;
  } else {
    b0 = t.iblo[q];
    b1 = t.ibhi[q];
  }
}

}  // namespace almbm
