// Host-side declarations of the kernel launchers (defined in the .hip files).
#pragma once

#include "kernels.hpp"

namespace almbm {

// Hub-row neighbour sums of C X into out (no-op when C has no hubs).
// lb: the L-BFGS rings (empty: gradient descent).  With rings, the row kernels
// step along the ring's current direction E instead of G and the gradient
// passes write y_k = G_new - G_old (ring type RingT<T>); the line-search
// product (instantiated for the ring type) multiplies E.
template <typename T>
void launch_hub_rows(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* X,
                     typename Acc<T>::type* out, const DevScalars* sc, int refresh_every, hipStream_t st,
                     const LbfgsRing<T>& lb = LbfgsRing<T>{});
template <typename T>
void launch_objgrad_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* R, const double* y,
                         const double* b, double sigma, T* G, double* Av, double* part, const DevScalars* sc,
                         int refresh_every, const BlockTab& tab, int nblk, hipStream_t st,
                         const LbfgsRing<RingT<T>>& lb = LbfgsRing<RingT<T>>{});
template <typename T>
void launch_quadq_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* G,
                       typename Acc<T>::type* Q, double* part, const DevScalars* sc, const BlockTab& tab, int nblk,
                       hipStream_t st, const LbfgsRing<T>& lb = LbfgsRing<T>{});
template <typename T>
void launch_upd_eval_diag(long n, int r, int variant, T* R, T* G, const typename Acc<T>::type* Q, const double* y,
                          const double* b, double sigma, double* Av, double* part, const DevScalars* sc,
                          int refresh_every, const BlockTab& tab, int nblk, hipStream_t st,
                          const LbfgsRing<RingT<T>>& lb = LbfgsRing<RingT<T>>{});
// L-BFGS steps (lbfgs_kernels.hip).  Reset at the start of a subproblem.
// Empty memories of m pairs for `count` instances (states s[0..count)).
void launch_lbfgs_reset(LbfgsState* s, int m, hipStream_t st, int count = 1);
// Inner products of the new gradient G and of y_k with the stored vectors
// (len = n*r elements each without a table; with one, the rows of each block
// at width r), per block of nb blocks into part[slot][kLbfgsDots].
template <typename T>
void launch_lbfgs_dots(long len, int r, const T* G, const LbfgsRing<RingT<T>>& lb, double* part, int nb,
                       const DevScalars* sc, hipStream_t st, const BlockTab& tab = BlockTab{});
// Pair update and the coefficients of the next direction (one block per instance).
void launch_fin_lbfgs(const double* part, int nb, const DevScalars* sc, LbfgsState* s, hipStream_t st,
                      const BlockTab& tab = BlockTab{}, int count = 1);
// E = cg G + sum (ce E_a + cy y_a) into the current slot, and the quartic's
// direction-dependent partial sums along -E (NUM_P per block).
template <typename T>
void launch_lbfgs_combine(long n, int r, int variant, const T* R, const T* G, const double* y, const double* b,
                          double sigma, const double* Av, const LbfgsRing<RingT<T>>& lb, double* part,
                          const DevScalars* sc, int nblk, hipStream_t st, const BlockTab& tab = BlockTab{});
// Direction-dependent totals of the quartic from the combine partials (one block per instance).
void launch_fin_lsdir(const double* part, int nb, DevScalars* sc, LbfgsState* s, hipStream_t st,
                      const BlockTab& tab = BlockTab{}, int count = 1);
template <typename T>
void launch_quad_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* G, double* part,
                      const DevScalars* sc, int nblk, hipStream_t st);
template <typename T>
void launch_ls_diag(const Cost<typename Acc<T>::type>& C, int r, int variant, const T* R, const T* G,
                    const double* y, const double* b, double* part, int nblk, hipStream_t st);

template <typename T>
void launch_edges_p1(const EdgeAdj& A, long n, int r, int variant, const T* R, const double* y, const double* b,
                     double sigma, double* Av, double* wE, double* part, const DevScalars* sc, int nblk,
                     hipStream_t st, double rho = 1.0);
template <typename T>
void launch_edges_p2(const Cost<typename Acc<T>::type>& C, const EdgeAdj& A, int r, int variant, const T* R,
                     const double* wE, double c_tr, double j_coef, const T* G_in, T* G, double* part,
                     const DevScalars* sc, int nblk, hipStream_t st);
template <typename T>
void launch_edges_p3(const Cost<typename Acc<T>::type>& C, const EdgeAdj& A, int r, int variant, const T* R,
                     const T* G, const double* y, const double* b, const double* Av, double* part,
                     const DevScalars* sc, int nblk, hipStream_t st, double rho = 1.0);
// part2 (64 x (NUM_P + kMaxR) doubles, nullable): the finalizers first reduce
// the nb partial rows to 64 with 64 blocks, then finish with one block.
void launch_fin_edges1(const double* part, int nb, int r, DevScalars* sc, const double* y, const double* b,
                       double sigma, double c_tr, double* Av, hipStream_t st, double* part2 = nullptr);
void launch_fin_edges2(const double* part, int nb, int r, DevScalars* sc, double sigma, int mode, double* f_out,
                       hipStream_t st, double* part2 = nullptr);
void launch_fin_edges3(const double* part, int nb, int r, DevScalars* sc, const double* y, const double* b,
                       double sigma, double c_tr, double j_coef, int mode, double* coeffs_out, double* t_out,
                       hipStream_t st, double* part2 = nullptr);

void launch_fin_objgrad(const double* part, int nb, DevScalars* sc, double sigma, int mode, double* f_out,
                        hipStream_t st, const BlockTab& tab = BlockTab{}, int count = 1);
void launch_fin_step(const double* part_c2, int nb, int c2_stride, DevScalars* sc, double sigma, double j_extra,
                     int mode, double* coeffs_out, double* t_out, hipStream_t st, const BlockTab& tab = BlockTab{},
                     int count = 1);
void launch_dual_batch(long m, const double* Av, const double* b, const double* y_in, double* y_out, double sigma,
                       double* part, DevScalars* sc, const double* bnorms, const BlockTab& tab, int nb, int count,
                       hipStream_t st);
void launch_inner_reset_batch(DevScalars* sc, int count, const double* tols, const int32_t* active, int max_inner,
                              int step_rule, double eta, hipStream_t st);
void launch_copy_active(long m, const double* src, double* dst, const int32_t* active, const BlockTab& tab, int nb,
                        hipStream_t st);
template <typename T>
void launch_fill_column(long n, int rs, T* R, const double* v, const int32_t* col, const double* scale,
                        const BlockTab& tab, int nb, hipStream_t st);
void launch_fin_ls(const double* part, int nb, DevScalars* sc, double sigma, double* coeffs_out, double* t_out,
                   hipStream_t st);
template <typename T>
void launch_update(long len, T* R, const T* G, const DevScalars* sc, int use_flag, hipStream_t st);
int dual_blocks(long m);
// y_out = y_in - sigma (Av - b) on row 0 and - sigma_tail (Av - b) on the other
// rows (sigma_tail <= 0: sigma everywhere).
void launch_dual(long m, const double* Av, const double* b, const double* y_in, double* y_out, double sigma,
                 double* part, DevScalars* sc, double bnorm, double* pinf_out, hipStream_t st,
                 double sigma_tail = 0.0);
void launch_inner_reset(DevScalars* sc, double tol, int max_inner, int step_rule, double eta, hipStream_t st);
template <typename T>
void launch_set_column(long n, int rs, int c, T* R, const double* v, double scale, hipStream_t st);
template <typename T>
void launch_restride_batch(const BlockTab& tab, int nb, const T* src, T* dst, const int64_t* ob, const int32_t* os,
                           const int64_t* nbase, const int32_t* ns, const int32_t* nc, hipStream_t st);
template <typename T>
void launch_relayout(long n, int ss, int nc, int rd, const T* src, T* dst, const double* v, double scale,
                     hipStream_t st);
template <typename S, typename D>
void launch_convert(long len, const S* src, D* dst, hipStream_t st);

int vec_blocks(long n);
void launch_slack_mv(const Cost<double>& C, int cons_kind, const EdgeAdj& A, const double* y, double c_tr,
                     double j_coef, const DevScalars* sc, const double* x, double* out, hipStream_t st);
void launch_slack_mv_tab(const Cost<double>& C, const double* y, const double* x, double* out, const BlockTab& tab,
                         int nb, hipStream_t st);
void launch_dots(long n, int ncol, const double* Q, long ldq, const double* w, double* part, int pstride, int nb,
                 double* h, hipStream_t st, const VecBatch& vb = VecBatch{});
void launch_sub(long n, int ncol, const double* Q, long ldq, const double* h, double* w, double* part, int nb,
                hipStream_t st, const VecBatch& vb = VecBatch{});
void launch_fin_ab(const double* part, int nb, const double* h1, const double* h2, int j, double* alpha, double* beta,
                   hipStream_t st, const VecBatch& vb = VecBatch{});
void launch_scale(long n, const double* w, const double* beta, double* q, double* part, int nb, double* qsum,
                  hipStream_t st, const VecBatch& vb = VecBatch{}, int bstride = 0);
void launch_gather_flags(const DevScalars* sc, int count, int32_t* out, hipStream_t st);
void launch_fin_sum(const double* part, int nb, double* out, int do_sqrt, hipStream_t st,
                    const VecBatch& vb = VecBatch{}, int ostride = 0);
void launch_rand(long n, uint64_t seed, double* x, double* part, int nb, hipStream_t st,
                 const VecBatch& vb = VecBatch{});
// x <- v + eps x / ||x|| per instance (norms[inst * nstride]), partial ||x||^2.
void launch_mix(long n, double eps, const double* v, double* x, const double* norms, int nstride, double* part,
                int nb, hipStream_t st, const VecBatch& vb = VecBatch{});
// Fourth moments of q <= 8 directions (V n x q column-major) per block of the
// nb-block grid: part[b * ne + e], ne = np (np + 1) / 2, np = q (q + 1) / 2.
void launch_gram4(long n, int q, const double* V, double* part, int nb, hipStream_t st);
// The edge-row moments of the trace + edge family (edges ei[e] < ej[e], E of them).
void launch_gram4_edges(long E, long n, int q, const int32_t* ei, const int32_t* ej, const double* V, double* part,
                        int nb, hipStream_t st);
// v = sum_{c < ncol} Q[:, c] s[c] (per instance s + inst * hstride; with
// ncols, at most ncols[inst] columns), partial ||v||^2.
void launch_combine(long n, int ncol, const double* Q, long ldq, const double* s, double* v, double* part, int nb,
                    hipStream_t st, const VecBatch& vb = VecBatch{}, const int32_t* ncols = nullptr);
void launch_resid(long n, const double* z, const double* v, double theta, const double* thetas, double* part, int nb,
                  hipStream_t st, const VecBatch& vb = VecBatch{});
void launch_quartic_norm(long n, int cons_kind, const EdgeAdj& A, const double* x, double* part, int nb,
                         hipStream_t st, const VecBatch& vb = VecBatch{});

void launch_ws_features(const Cost<double>& C, float* F, float* ldeg, hipStream_t st);
int ws_param_count(int nin, int h);
bool launch_ws_forward(const float* P, int nin, int h, const float* mu, const float* isd, long n, const float* X,
                       double* out, hipStream_t st);
void launch_ws_pool(const float* F, long n, double* part, int nb, double* out, hipStream_t st);
bool launch_ws_backward(const float* P, int nin, int h, const float* mu, const float* isd, long n, const float* X,
                        const float* T, float* gpart, double* lpart, int nb, float* grad, double* loss,
                        hipStream_t st);
void launch_ws_adam(float* P, const float* g, float* m, float* v, int np, float lr, float b1, float b2, float eps,
                    int step, hipStream_t st);

}  // namespace almbm
