// Launchers of the kernels beyond the plain rate path: the polar long-range
// factor, group velocities, the phonon-linewidth reduction, Philox streams,
// network initialisation, training-set selection, row gathers, the
// finiteness scan and the 3-phonon coupling contractions.
#pragma once

#include "common.hpp"

namespace phx {

// Born charges (device [nat, 3, 3]) and the rest of a polar crystal's data.
struct PolarDev {
    const double* born;
    double eps[9];
    double alpha;
    int g_max;
    int nat;
};

// L[p, nu] = pref sum_sa D_sa(q_p) E[p, nu, sa], D_{s b}(q) = sum_{G: q+G != 0}
// w(q+G) sum_a K_a Z*_{s, a b}, w(K) = e^{-K.eps.K/(4 alpha)} / (K.eps.K), K = 2 pi (q+G).
// Points: fractional coordinates (frac) or every point of mesh m (frac == nullptr).
hipError_t launch_polar_factor(const double* frac, Mesh m, int64_t np, const cd* E, int nm,
                               const PolarDev& pd, cd* L, hipStream_t s);

// g[q, nu, n, m] += i L[q, nu] [U_k^dagger U_{k+q}]_{n m} for the q of one k
// (U_k [nW, nW] and U_{k+q} [nq, nW, nW] with eigenvectors as columns).
hipError_t launch_polar_add_g(cd* g, int64_t nq, const cd* Uk, const cd* Ukq, const cd* L,
                              int nW, int nm, hipStream_t s);

// Pv[p, a, r] = i R_a(r) P[p, r] (the phase table of the k-derivative).
hipError_t launch_velocity_phases(const cd* P, int64_t np, const int32_t* R, int nR, cd* Pv,
                                  hipStream_t s);
// v[p, b, a] from dH [p, 3, nW, nW] and U [p, nW, nW] (columns; transposed = U[p, band,
// orbital] when u_transposed): diagonal of U^dagger dH_a U, degenerate groups
// (|d eps| < tol) diagonalised.  *bad is set to 1 when a group exceeds 8 bands.
hipError_t launch_group_velocities(const cd* dH, const cd* U, bool u_transposed,
                                   const double* eps, int64_t np, int nW, double tol, double* v,
                                   int32_t* bad, hipStream_t s);
// Per-axis maximum of |v| over a velocity table [np, nW, 3] -> vmax[3].
hipError_t launch_velocity_max(const double* v, int64_t np, int nW, double* vmax, hipStream_t s);

// Linewidth partials -> acc[q, nu] (+=), states in order.  Factorised layout:
// lw[st, line, q0, nu] for the (state, line) pairs with line_bands != 0, q = q0 NL +
// line.  Direct layout: lw[st, q, nu].
hipError_t launch_lw_reduce_lines(const double* lw, const uint32_t* line_bands,
                                  const uint32_t* live, int nst, int NL, int N0, int nm,
                                  double* acc, hipStream_t s);
hipError_t launch_lw_reduce_dense(const double* lw, int nst, int64_t N, int nm, double* acc,
                                  hipStream_t s);
// P = scale n (n + 1) omega acc for omega >= omega_min, else 0.
hipError_t launch_lw_finish(const double* acc, const double* omega, const double* nb, int64_t n,
                            double omega_min, double scale, double* P, hipStream_t s);

// Philox-4x64-10 streams (see the header).
hipError_t launch_philox_uniform(uint64_t seed, uint64_t offset, int64_t n, double* out,
                                 hipStream_t s);
hipError_t launch_philox_randint(uint64_t seed, uint64_t offset, int64_t n, int64_t hi,
                                 int32_t* out, hipStream_t s);
// params[off + j] = (2 u_{off+j} - 1) / div for j < count (float or double).
hipError_t launch_uniform_fill(void* params, bool f64, uint64_t seed, int64_t off, int64_t count,
                               double div, hipStream_t s);

// Training-set selection (see phoebe_gpu_training_set).
constexpr int kTsBlocks = 1024;  // fixed grid of the statistics pass (fixed summation order)
hipError_t launch_ts_state_max(const double* D, int64_t ns, int64_t per, double* dmax,
                               hipStream_t s);
// stats[0] = selected count (as double, exact below 2^53), stats[1] = sum of T/D.
hipError_t launch_ts_stats(const double* T, const double* D, const double* dmax, int64_t ns,
                           int64_t per, double thr, double* partial, double* stats,
                           hipStream_t s);
constexpr int kTsChunk = 4096;
hipError_t launch_ts_count(const double* D, const double* dmax, int64_t ns, int64_t per, double thr,
                           uint64_t seed, double p_keep, int32_t* counts, hipStream_t s);
// in-place exclusive scan of n int32 counts; total in *total
hipError_t launch_exclusive_scan(int32_t* counts, int64_t n, int64_t* total, hipStream_t s);
hipError_t launch_ts_write(const double* T, const double* D, const double* dmax, int64_t ns,
                           int64_t per, int nm, int64_t nq, double thr, uint64_t seed,
                           double p_keep, double c, const int32_t* offsets, int64_t cap,
                           int32_t* o_state, int32_t* o_q, int32_t* o_nu, float* o_y,
                           hipStream_t s);

hipError_t launch_gather_rows32(const uint32_t* src, int64_t words, const int32_t* idx, int64_t n,
                                uint32_t* dst, hipStream_t s);

// *flag |= 1 if any of the n doubles is NaN or infinite.
hipError_t launch_nonfinite(const double* x, int64_t n, int32_t* flag, hipStream_t s);

// 3-phonon coupling helpers.
hipError_t launch_real_to_complex(const double* x, int64_t n, cd* out, hipStream_t s);
// out[p] = -(q[i] + qp[j]) for p = i nqp + j
hipError_t launch_neg_pair_sum(const double* q, int64_t nq, const double* qp, int64_t nqp,
                               double* out, hipStream_t s);
// T[i, r, nu, bc] = sum_sa S[i, r, sa, bc] conj(E1[i, nu, sa]), bc < nm^2
hipError_t launch_v3_fold(const cd* S, int64_t nq, int nr, int nm, const cd* E1, cd* T,
                          hipStream_t s);
// Y[j, nu, nu', c] = sum_b X[j, nu, b, c] conj(E2[j, nu', b])
hipError_t launch_v3_rot1(const cd* X, int64_t nqp, int nm, const cd* E2, cd* Y, hipStream_t s);
// V[j, nu, nu', nu''] = sum_c Y[j, nu, nu', c] conj(E3[j, nu'', c])
hipError_t launch_v3_rot2(const cd* Y, int64_t nqp, int nm, const cd* E3, cd* V, hipStream_t s);

}  // namespace phx
