// Persistent multi-system rate kernel (batched form), FP32 contractions.
#pragma once

#include "lowp.hpp"

namespace phx {

constexpr int kMBB = 8;  // final bands per rotation pass

// Everything one system's tasks read (device pointers).
struct SysDesc {
    const cf* F;               // [states][rp_pad][nc_pad]
    int rp_pad, nc_pad, n_rp, rmax;
    int nW, nm, tq, tn;
    const int32_t* rp_packed;  // [n_rp]
    Mesh mesh;
    int64_t nq;
    const int32_t* st_kmesh;
    const int32_t* st_band;
    const int32_t* st_mlo;
    const int32_t* st_mhi;
    const double* eps;
    const double* focc;
    const double* omega;
    const double* nb;
    const cd* U;  // transposed: U[k, band, orbital]
    const cd* E;
    double sigma;
    double* partial;           // [states][n_qtiles]
    int n_qtiles;
};

struct BTask {
    int sys, state, qtile, pad;
};

bool batched_tile_supported(int tq, int tn);
size_t batched_lds(int tq, int rmax, int rp_pad, int nc_pad, int nm);
hipError_t prepare_batched_rates(size_t lds);
hipError_t launch_batched_rates(const SysDesc* sys, const BTask* tasks, int n_tasks, int* head,
                                int n_wg, size_t lds, hipStream_t s);

}  // namespace phx
