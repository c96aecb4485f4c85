// Learned-proposal launchers (MLP training/inference, sampler).
#pragma once

#include "kernels.hpp"

namespace phx {

// with act set, silu(C) is also written to act (same leading dimension)
template <class T>
hipError_t launch_mlp_gemm(bool ta, bool tb, const T* A, int64_t lda, const T* B, int64_t ldb, T* C,
                           int64_t ldc, int64_t M, int64_t N, int64_t K, const T* bias, int acc,
                           hipStream_t s, T* act = nullptr);
template <class T>
hipError_t launch_silu_fwd(const T* z, T* a, int64_t n, hipStream_t s);
template <class T>
hipError_t launch_silu_bwd(const T* da, const T* z, T* dz, int64_t n, hipStream_t s);
template <class T>
hipError_t launch_mse_grad(const T* y, const T* t, T* dy, int64_t B, double* sums, int nblk,
                           hipStream_t s);
template <class T>
hipError_t launch_colsum(const T* dz, int64_t B, int64_t N, T* db, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int t, double lr,
                       double b1, double b2, double eps, hipStream_t s);
template <class T>
hipError_t launch_features(const int32_t* k_idx, const double* eps, const int32_t* q_idx,
                           const int32_t* nu, int64_t B, Mesh mesh, int nm, int n_harm, double e0,
                           double escale, T* X, hipStream_t s);
int feature_count(int nm, int n_harm);
hipError_t launch_proposal_raw(const float* y, int64_t nq, int nm, double c, double* p,
                               hipStream_t s);
hipError_t launch_weight_list(const double* D, const int32_t* list, const float* y, int64_t n,
                              double* E, hipStream_t s);
hipError_t launch_sum_modes(const double* E, int64_t N, int nm, double* p, hipStream_t s);
hipError_t launch_sample(double* p, int64_t N, double mix, const double* u, int S, int32_t* q_idx,
                         double* q_w, int64_t nk, hipStream_t s);
// entries f = k NR + r of D [nk, NR] with D > thr dmax[k], in flat order; counts has
// select_rows_chunks(nk, NR) entries, total_out one (device)
hipError_t launch_select_rows(const double* D, const double* dmax, int64_t nk, int64_t NR,
                              double thr, int32_t* counts, int64_t* total_out, int32_t* list,
                              hipStream_t s);
int64_t select_rows_chunks(int64_t nk, int64_t NR);
hipError_t launch_features_flat(const int32_t* kmesh, const double* epsk, const int32_t* list,
                                int64_t n, int64_t NR, Mesh mesh, int nm, int n_harm, double e0,
                                double escale, float* X, hipStream_t s);

}  // namespace phx
