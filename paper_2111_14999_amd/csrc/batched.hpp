// Persistent multi-system rate kernel (batched form), FP32 contractions.
#pragma once

#include "lowp.hpp"

namespace phx {

// One system of the batched form: the arguments of its rate tiles (device
// pointers: F [states][rp_pad][nc_pad], tables, state lists, partials) and the
// tile shape (TQ, TN) the autotuner chose for it.
struct SysDesc {
    RateArgsLP a;
    int tq, tn;
};

struct BTask {
    int sys, state, qtile, pad;
};

// The tile shapes (TQ, TN) of the persistent kernels, one kernel per shape;
// shape index of (tq, tn), or -1.  nc = nModes*nW stage-2 columns fit one
// column pass when 64*TN >= nc.
constexpr int kBatchedShapes = 12;
int batched_shape(int tq, int tn);
bool batched_tile_supported(int tq, int tn, int nc);
// dynamic LDS of a system's tiles, with or without the staged rotation operands
size_t batched_lds(int tq, int rmax, int rp_pad, int nc_pad, int nm, int nW, bool stage);
// staging pays for the shape's kernel at these LDS sizes (see lp_stage_pays)
bool batched_stage_pays(int shape, size_t lds0, size_t lds1);
// sets the kernel's dynamic LDS limit (outside a stream capture)
hipError_t prepare_batched_rates(int shape, size_t lds);
hipError_t launch_batched_rates(int shape, const SysDesc* sys, const BTask* tasks, int n_tasks,
                                int* head, int n_wg, size_t lds, hipStream_t s);

}  // namespace phx
