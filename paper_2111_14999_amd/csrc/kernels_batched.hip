// Batched form: persistent kernels drain a work queue of (system, state, q tile)
// tasks over many independent systems of different sizes.
//
// A task is the fused FP32 rate tile of the one-system path (stage2_lp_tile:
// X[q, sa*nW + b] = sum_Rp e^{i2pi q.Rp} F[Rp, sa*nW + b] on
// v_mfma_f32_16x16x4f32 for 16*TQ q points, the U_{k+q} and phonon rotations in
// FP32, the smeared rate terms in FP64 into partial[state, q tile]), at the
// system's own (TQ, TN).  There is one persistent kernel per tile shape, each
// with its own queue: a kernel holds exactly the registers of its shape, so a
// wide shape does not lower the occupancy of the narrow ones.
#include "batched.hpp"
#include "stage2_lp_tile.hpp"

namespace phx {

// Waves per SIMD a shape's kernel is compiled for: three where its registers fit
// without spills, two for the widest tiles.
constexpr int batched_waves_per_simd(int tq, int tn) { return tn >= 8 || tq * tn >= 8 ? 2 : 3; }

// Every work-group loops: take the next task index from the queue head, run
// it, stop when the queue is exhausted (every wave reaches the exit).
//
// No branch on the thread id encloses the queue fetch or the tile's result
// store: the whole of wave 0 (a wave-uniform branch) takes the task, lane 0
// adding 1 and the other lanes 0, so the compiler cannot join the store at the
// end of one task with the fetch of the next into one thread-divergent path,
// which would put the work-group's barriers under a divergent loop.
template <int TQ, int TN>
__global__ __launch_bounds__(256, batched_waves_per_simd(TQ, TN)) void batched_rates_kernel(const SysDesc* __restrict__ sys,
                                                               const BTask* __restrict__ tasks,
                                                               int n_tasks, int* head) {
    extern __shared__ char smem_raw[];
    __shared__ LpShared sh;
    __shared__ int s_task;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (;;) {
        if (wave == 0) {
            const int old = atomicAdd(head, (threadIdx.x & 63) == 0 ? 1 : 0);
            s_task = __builtin_amdgcn_readfirstlane(old);  // lane 0's value
        }
        __syncthreads();
        // the task index is the same for the whole work-group: with it marked uniform,
        // the task and its system's arguments load into scalar registers
        const int t = __builtin_amdgcn_readfirstlane(s_task);
        __syncthreads();
        if (t >= n_tasks) break;
        const BTask tk = tasks[t];
        const int sid = __builtin_amdgcn_readfirstlane(tk.sys);
        const int state = __builtin_amdgcn_readfirstlane(tk.state);
        const int qtile = __builtin_amdgcn_readfirstlane(tk.qtile);
        const RateArgsLP a = sys[sid].a;
        stage2_lp_tile<PHOEBE_FP32, TQ, TN>(a, state, qtile, smem_raw, sh);
    }
}

namespace {

// the shapes, in the order of their shape index
constexpr int kShapes[kBatchedShapes][2] = {{1, 1}, {2, 1}, {1, 2}, {2, 2}, {1, 3}, {2, 3},
                                             {1, 4}, {2, 4}, {1, 6}, {1, 8}, {1, 12}, {1, 16}};

template <int I>
const void* shape_fn() {
    return reinterpret_cast<const void*>(batched_rates_kernel<kShapes[I][0], kShapes[I][1]>);
}

const void* kernel_of(int shape) {
    switch (shape) {
        case 0: return shape_fn<0>();
        case 1: return shape_fn<1>();
        case 2: return shape_fn<2>();
        case 3: return shape_fn<3>();
        case 4: return shape_fn<4>();
        case 5: return shape_fn<5>();
        case 6: return shape_fn<6>();
        case 7: return shape_fn<7>();
        case 8: return shape_fn<8>();
        case 9: return shape_fn<9>();
        case 10: return shape_fn<10>();
        case 11: return shape_fn<11>();
        default: return nullptr;
    }
}

size_t g_lds_set[kBatchedShapes] = {};

}  // namespace

int batched_shape(int tq, int tn) {
    for (int i = 0; i < kBatchedShapes; ++i)
        if (kShapes[i][0] == tq && kShapes[i][1] == tn) return i;
    return -1;
}

bool batched_tile_supported(int tq, int tn, int nc) {
    return 64 * tn >= nc && batched_shape(tq, tn) >= 0;
}

size_t batched_lds(int tq, int rmax, int rp_pad, int nc_pad, int nm, int nW, bool stage) {
    return stage2_lp_lds(PHOEBE_FP32, tq, rmax, rp_pad, nc_pad, nm, nW, stage);
}

bool batched_stage_pays(int shape, size_t lds0, size_t lds1) {
    const void* fn = kernel_of(shape);
    return fn && lp_stage_pays(fn, lds0, lds1);
}

hipError_t prepare_batched_rates(int shape, size_t lds) {
    const void* fn = kernel_of(shape);
    if (!fn || lds > 160 * 1024 - 1024) return hipErrorInvalidValue;
    if (lds <= g_lds_set[shape]) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) g_lds_set[shape] = lds;
    return e;
}

hipError_t launch_batched_rates(int shape, const SysDesc* sys, const BTask* tasks, int n_tasks,
                                int* head, int n_wg, size_t lds, hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    hipError_t e = prepare_batched_rates(shape, lds);
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&sys, (void*)&tasks, (void*)&n_tasks, (void*)&head};
    e = hipLaunchKernel(kernel_of(shape), dim3(n_wg), dim3(256), args, lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace phx
