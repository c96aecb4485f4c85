// Reduced-precision (FP32 / split-BF16) launchers.
#pragma once

#include "kernels.hpp"

namespace phx {

constexpr int kMBLP = 8;  // final bands per rotation pass

struct RateArgsLP {
    const void* F;             // FP32: cf [nst, rp_pad, nc_pad]; BF16: u16 [nst, 2NP, nc_pad, rp_pad]
    int rp_pad, nc_pad;
    int n_rp;
    const int32_t* rp_packed;
    int rmax;
    Mesh mesh;
    int64_t nq_mesh;
    const int32_t* st_kmesh;
    const int32_t* st_band;
    const int32_t* st_row;
    const int32_t* st_mlo;
    const int32_t* st_mhi;
    const int64_t* q_off;
    const int32_t* q_idx;
    const double* q_w;
    const double* eps;
    const double* focc;
    const cd* U;
    const double* omega;
    const double* nb;
    const cd* E;
    int nW, nm;
    double sigma;
    double* partial;
    int n_qtiles;
    // stage each rotation chunk's U_{k+q} rows and E_q in LDS (set by the launcher
    // where the larger LDS block costs no occupancy)
    int stage;
};

// C (cf) = A (cd phases) * B in the given precision (FP32, BF16X3, BF16X6).
hipError_t launch_cgemm_lp(int prec, const cd* A, int64_t lda, const cd* B, int64_t ldb, cf* C,
                           int64_t ldc, int64_t M, int64_t N, int K, hipStream_t s);
hipError_t launch_cgemm_lp_cf(int prec, const cd* A, int64_t lda, const cf* B, int64_t ldb, cf* C,
                              int64_t ldc, int64_t M, int64_t N, int K, hipStream_t s);
hipError_t launch_fold_uk_lp(int prec, const cf* G, int64_t ldg, const cd* U,
                             const int32_t* st_row, int row0, const int32_t* st_kmesh,
                             const int32_t* st_band, int nst, int n_rp, int nm, int nW, int cw,
                             int rp_pad, int nc_pad, void* F, hipStream_t s);
hipError_t launch_stage2_rates_lp(int prec, const RateArgsLP& a, int nst, hipStream_t s);
size_t stage2_lp_lds(int prec, int tq, int rmax, int rp_pad, int nc_pad, int nm, int nW,
                     bool stage);
// staging in LDS pays for a kernel when its larger LDS block (shm1) allows as many
// resident work-groups per CU as the smaller one (shm0)
bool lp_stage_pays(const void* kern, size_t shm0, size_t shm1);
int stage2_lp_config(int nm, int nW, int* tq_out, int* tn_out);
hipError_t launch_fold_all_lp(const cf* G, const cd* U, int n_rp, int nm, int nW, cf* F,
                              hipStream_t s, int64_t ldf = -1);
hipError_t launch_rotate_g_lp(const cf* X, int64_t nq, const cd* Ukq, const cd* E, int nW, int nm,
                              cd* g, hipStream_t s);

}  // namespace phx
