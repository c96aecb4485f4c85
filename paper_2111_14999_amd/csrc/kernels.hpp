// Launchers of the library's HIP kernels (host side).  All return hipError_t of
// the launch; shapes are validated by the caller before any launch.
#pragma once

#include "common.hpp"

namespace phx {

// P[p, r] = e^{i 2 pi x_p . R_r}.  Points are either fractional coordinates
// (frac != nullptr, [np, 3]) or mesh points given by linear index (idx, or
// 0..np-1 when idx == nullptr) of mesh m.  R packed as int3 on device.
hipError_t launch_phase_table(const double* frac, const int32_t* idx, Mesh m, int64_t np,
                              const int32_t* R, int nR, cd* P, int64_t ldp, hipStream_t s);

// C[M, N] = A[M, K] * B[K, N], complex FP64 on MFMA.  Row-major with leading
// dimensions (in complex elements).
hipError_t launch_zgemm(const cd* A, int64_t lda, const cd* B, int64_t ldb, cd* C, int64_t ldc,
                        int64_t M, int64_t N, int K, hipStream_t s);

// Real force constants -> complex mass-weighted Phi(R)/sqrt(M_s M_s').
hipError_t launch_mass_weight(const double* phi, const double* mass, int nR, int nm, cd* out,
                              hipStream_t s);

// In-place batched Hermitian eigensolver (cyclic Jacobi, FP64).  A [batch, n, n]
// is destroyed; w [batch, n] ascending; V [batch, n, n] eigenvectors as columns.
hipError_t launch_eig_herm(cd* A, int n, int64_t batch, double* w, cd* V, hipStream_t s);

// Phonon post-processing: omega = C_OMEGA sqrt(max(lam, 0)); e[q, sa, nu] =
// z[q, sa, nu] l_{s, q nu} (0 when omega < omega_min); nb Bose occupation
// (0 when inactive or kT <= 0).
hipError_t launch_phonon_post(const double* lam, const cd* z, const double* mass, int nat,
                              int64_t nq, double omega_min, double kT, double* omega, cd* e,
                              double* nb, hipStream_t s);

// Fermi occupations of a band table.
hipError_t launch_fermi(const double* eps, int64_t n, double mu, double kT, double* f,
                        hipStream_t s);

// Window: mask[k, b] = win_lo < eps[k, b] < win_hi; flag[k] = any(mask[k, :]).
hipError_t launch_window(const double* eps, int64_t nk, int nW, double lo, double hi,
                         uint8_t* mask, int32_t* flag, hipStream_t s);

// Ordered compaction of flags: out[j] = j-th index with flag != 0; *count on device.
hipError_t launch_compact(const int32_t* flag, int64_t n, int32_t* out, int32_t* count,
                          hipStream_t s);

// Per-band min/max over a band table and the maximum phonon energy.
hipError_t launch_band_extrema(const double* eps, int64_t nk, int nW, const double* omega,
                               int64_t nq, int nm, double* bmin, double* bmax, double* wmax,
                               hipStream_t s);

// In-place transpose of count n x n complex matrices.
hipError_t launch_transpose_batch(cd* U, int64_t count, int n, hipStream_t s);

// Stage-1 fold: F[st, r, sa*nW + b] = sum_a conj(U_k[a, n]) G[kb, r, sa, a, b]
// for each state st = (kb, n); rows r >= n_rp and columns >= NC are zero.
// Zeroes the padding of F (rows n_rp.., columns ncol..), which the folded stage 1
// does not write.
hipError_t launch_zero_fpad(void* F, int64_t nst, int rp_pad, int nc_pad, int n_rp, int ncol,
                            int esize, hipStream_t s);
hipError_t launch_fold_uk(const cd* G, int64_t ldg, const cd* U, const int32_t* st_krow,
                          int row0, const int32_t* st_kmesh, const int32_t* st_band, int nst, int n_rp,
                          int nm, int nW, int cw, int rp_pad, int nc_pad, cd* F, hipStream_t s);

struct RateArgs {
    const cd* F;            // [nst, rp_pad, nc_pad]
    int rp_pad, nc_pad;
    int n_rp;
    const int32_t* rp_packed;  // [n_rp] (R0+r) | (R1+r)<<8 | (R2+r)<<16
    int rmax;
    Mesh mesh;
    int64_t nq_mesh;
    const int32_t* st_kmesh;   // [nst] mesh index of the state's k
    const int32_t* st_band;    // [nst]
    const int32_t* st_row;     // [nst] evaluated-k row of the state
    const int32_t* st_mlo;     // [nst] first final band to sum
    const int32_t* st_mhi;     // [nst] last final band to sum (inclusive)
    const int64_t* q_off;      // per row, or nullptr for full mesh
    const int32_t* q_idx;
    const double* q_w;
    const double* eps;         // [Nk, nW]
    const double* focc;        // [Nk, nW]
    const cd* U;               // [Nk, nW, nW] transposed: U[k, band, orbital]
    const double* omega;       // [Nq, nm]
    const double* nb;          // [Nq, nm]
    const cd* E;               // [Nq, nm, nm]: E[q, nu, sa] = z[q][sa][nu] l_{sa,nu}
    int nW, nm;
    double sigma;
    double* partial;           // [nst, n_qtiles]
    int n_qtiles;
    double* terms;             // nullable [nst, nq_mesh, nm]: per-(q, mode) terms, summed over m
    double terms_scale;        // factor applied to each stored term
    // factorised full-mesh form: X[q] = sum_R0 P0[q0, R0] T2[R0, q1 N2 + q2]
    const void* T2;            // [nst, W, N1*N2, nc_pad] of cd (FP64) or cf (FP32 form)
    const cd* P0;              // [N0, W]
    int W;                     // 2 rmax + 1
    int n_states;              // states of one launch (set by the launcher)
    const double* wmax;        // device scalar: largest phonon energy on the mesh
    const uint32_t* live;        // [nst, N1*N2, N0] live final bands of every point (line_live)
    const uint32_t* line_bands;  // [nst, N1*N2] union of a line's live bands, 0: none
    // extensions, FP64 forms only (all null/unused in the plain rate sum):
    const cd* Lpol;            // nullable [Nq, nm]: polar factor, g += i L(q,nu) [U_k^dag U_{k+q}]_nm
    const double* vel;         // nullable [Nk, nW, 3]: adaptive smearing from the group velocities,
                               // sigma_t = max(sigma, |ad_c . (v_nk - v_m,k+q)|), terms carry 1/sigma_t
    double ad_c[3];            // (A / sqrt 12) 2 pi / N_d per axis
    double* lw;                // nullable: phonon-linewidth partials of the launch's states
                               // (line kernel [st, line, q0, nu]; direct kernel [st, q, nu], zeroed)
    double inv_kT;             // 1 / kT (linewidth weight f (1 - f) / kT)
};

// Fused stage 2 (sum over Rp on MFMA) + rotations + rate terms.
hipError_t launch_stage2_rates(const RateArgs& a, int nst, hipStream_t s);

// Per-axis phase tables P[d][n, r] = e^{i2pi (n (r - rmax) mod N_d)/N_d}, [N0+N1+N2, W].
hipError_t launch_axis_phases(Mesh m, int rmax, cd* P, hipStream_t s);
// T1 (axis 2) and T2 (axis 1) of the factorised full-mesh sum over Rp.
// line_any (nullable): [nst, N1*N2]; T2 of a line whose entry is 0 is not formed.
hipError_t launch_axis_transforms(const cd* F, int rp_pad, int nc_pad, const int32_t* box_rp,
                                  int rmax, Mesh m, const cd* P, int nst, const uint32_t* line_any,
                                  cd* T1, cd* T2, hipStream_t s);
// With line_any set, a box of width 1, 3, 5, 7 or 9 whose F slab (W^2 x 64 columns)
// fits 64 KB of LDS and nc_pad % 64 == 0, both axes run in one pass and T1 is not
// used (T1 may then be null); this tells which route a call takes.
bool axis_transforms_fused(int rmax, int nc_pad, bool f32);
hipError_t launch_axis_transforms_f32(const cf* F, int rp_pad, int nc_pad, const int32_t* box_rp,
                                      int rmax, Mesh m, const cd* P, int nst,
                                      const uint32_t* line_any, cf* T1, cf* T2, hipStream_t s);
// The last axis written out for q0 in [q0a, q0b) of one T2 [W, N1*N2, nc_pad]:
// X [(q0 - q0a) N1 N2 + line, c] (rows ldx apart, c < nc); P as for the transforms.
hipError_t launch_axis0_out(const cd* T2, Mesh m, int nc_pad, int nc, int rmax, const cd* P,
                            int q0a, int q0b, cd* X, int64_t ldx, hipStream_t s);
hipError_t launch_axis0_out_f32(const cf* T2, Mesh m, int nc_pad, int nc, int rmax, const cd* P,
                                int q0a, int q0b, cf* X, int64_t ldx, hipStream_t s);
// The last axis and the rotation of g on the full mesh in one pass (FP64, nW and
// nModes <= 16, box width 1 to 7): g [N, nModes, nW, nW] of one k from its T2
// [W, N1*N2, ncp] (columns (sa, n, b)), E [N, nModes, nModes], Ukq [N, nW, nW].
bool axis0_rotate_supported(int rmax, int nW, int nm);
hipError_t launch_axis0_rotate(const cd* T2, Mesh m, int ncp, int rmax, const cd* P,
                               const cd* E, const cd* Ukq, int nW, int nm, cd* g, hipStream_t s);
// Stage 1 factorised over the axes of the Re box for one batch of kept k.
// Device lists: d_k0 [d0] distinct k0; pair_k1 [d01] and pair_off [d0+1] the
// distinct (k0, k1) pairs grouped by k0; kp_off [d01+1], k_row, k_k2 [nb] the
// batch rows (and their k2) grouped by pair.
struct ReBatch {
    int d0, d01;
    const int32_t *d_k0, *pair_k1, *pair_off, *kp_off, *k_row, *k_k2;
    const int32_t* d_plane;  // T0 plane of each distinct k0 (all planes resident), else null
    // per row of k_row (16-byte aligned): k2, first state, end of the row's states, 0
    const int32_t* k_ent;
};
// With fo set (nW = 16), the pair and k steps apply the U_k fold of the rates at
// once and write F [states of the batch, rp_pad, nc_pad] (columns sa*16 + b)
// instead of G; T0 is then stored with each 16 x 16 (a, b) block transposed.
struct FoldOut {
    const int32_t* row_st;    // [rows of the batch + 1] first state of each batch row
    const int32_t* st_kmesh;  // [states of the batch] mesh index of the state's k
    const int32_t* st_band;   // [states of the batch]
    const cd* U;              // [Nk, nW, nW] eigenvectors, transposed: U[k, band, orbital]
    int nW, nm, n_rp, rp_pad, nc_pad;
    void* F;                  // cd (FP64) or cf (FP32 form)
};
hipError_t launch_re_axes(const cd* g, int64_t NC, const int32_t* box_re, int rmax, Mesh m,
                          const cd* P, const ReBatch& b, const FoldOut* fo, cd* T0, cd* G,
                          int64_t ldg, hipStream_t s);
hipError_t launch_re_axes_f32(const cd* g, int64_t NC, const int32_t* box_re, int rmax, Mesh m,
                              const cd* P, const ReBatch& b, const FoldOut* fo, cf* T0, cf* G,
                              int64_t ldg, hipStream_t s);
// The same two steps apart, with T0 held for every k0 plane of the call: the
// planes in one pass over g (tr: transposed (a, b) blocks, for the folded
// form), then the pair and k steps of each batch.
hipError_t launch_re_planes(const cd* g, int64_t NC, const int32_t* box_re, int rmax,
                            const cd* P, const int32_t* k0_list, int n, bool tr, cd* T0,
                            hipStream_t s);
hipError_t launch_re_planes_f32(const cd* g, int64_t NC, const int32_t* box_re, int rmax,
                                const cd* P, const int32_t* k0_list, int n, bool tr, cf* T0,
                                hipStream_t s);
hipError_t launch_re_pairs(const cd* T0, int64_t NC, int rmax, Mesh m, const cd* P,
                           const ReBatch& b, const FoldOut* fo, cd* G, int64_t ldg, hipStream_t s);
hipError_t launch_re_pairs_f32(const cf* T0, int64_t NC, int rmax, Mesh m, const cd* P,
                               const ReBatch& b, const FoldOut* fo, cf* G, int64_t ldg,
                               hipStream_t s);
size_t re_axes_lds(int rmax, bool f32);

// Axis 0 on MFMA + rotations + rate terms, one work-group per (state, q1, q2) line.
// Columns sa*16 + b (nW <= 16), nc_pad = 64 TN with 4 TN >= nModes.
// Live final bands of every (state, point) for the line kernel (nW <= 16),
// their union per (state, line) and, added to n_live[0] and n_live[1], the
// number of (state, line) pairs with a live band and of 16-point units; the
// partial sum a.partial[st, line] of a pair without a live band is set to 0
// here (the line kernel skips such pairs).
hipError_t launch_line_live(const RateArgs& a, int nst, uint32_t* live, uint32_t* line_bands,
                            uint32_t* n_live, hipStream_t s);
hipError_t launch_line_rates(const RateArgs& a, int nst, hipStream_t s);
hipError_t launch_line_rates_f32(const RateArgs& a, int nst, hipStream_t s);
size_t line_rates_lds(int W, int N0, int nm, bool f32, bool lw = false);
int line_rates_ncpad(int nm, int nW);  // -1 where the form does not apply

// gamma[row, band] = scale * sum_t partial[st, t]
hipError_t launch_reduce_partials(const double* partial, int nst, int ntiles,
                                  const int32_t* st_row, const int32_t* st_band, int nW,
                                  double scale, double* gamma, hipStream_t s);

// interp_g rotation: g[k, q, nu, n, m] from X[q, sa, n, b] of one k.
hipError_t launch_rotate_g(const cd* X, int64_t nq, const cd* Uk, const cd* Ukq, const cd* E,
                           int nW, int nm, cd* g, hipStream_t s);

// fold for interp_g (all bands n): F[r, sa, n, b] = sum_a conj(U[a, n]) G[r, sa, a, b]
// (F rows ldf elements apart; ldf < 0: nm nW^2)
hipError_t launch_fold_all(const cd* G, const cd* U, int n_rp, int nm, int nW, cd* F,
                           hipStream_t s, int64_t ldf = -1);

hipError_t launch_gather_rows(const uint8_t* mask, const int32_t* kept, int64_t rows, int nW,
                              int32_t* rowflag, uint8_t* mask_out, int32_t* kept_out,
                              hipStream_t s);
hipError_t launch_build_states(const int32_t* ids, int nst, int nW, const int32_t* kept,
                               const double* eps, const double* bmin, const double* bmax,
                               const double* wmax, double cut, int32_t* st_row, int32_t* st_band,
                               int32_t* st_kmesh, int32_t* st_mlo, int32_t* st_mhi,
                               hipStream_t s);
int stage2_config(int nm, int nW, int* tq_out, int* tn_out);

hipError_t launch_delta_weights(int nst, int64_t N, Mesh mesh, const int32_t* st_kmesh,
                                const int32_t* st_band, const int32_t* st_mlo,
                                const int32_t* st_mhi, const double* eps, const double* focc,
                                const double* omega, const double* nb, int nW, int nm, double sigma,
                                double omega_min, double scale, double* D, hipStream_t s);

// helpers
hipError_t launch_kq_points(const double* k, int64_t nk, const double* q, int64_t nq,
                            double* kq, hipStream_t s);
// eps_kq [nk, nq, nW], Ukq [nk, nq, nW, nW] of k = mesh point k_idx[i] and q = mesh
// point j from the mesh's eps [N, nW] and U [N, nW, nW]
hipError_t launch_gather_kq_bands(const double* eps, const cd* U, int nW, Mesh m,
                                  const int32_t* k_idx, int64_t nk, int64_t nq, double* eps_kq,
                                  cd* Ukq, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace phx
