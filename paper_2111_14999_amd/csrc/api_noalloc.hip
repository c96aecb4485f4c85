// The non-allocating variant of the rate path: the same computation as
// phoebe_gpu_scatter_rates with its workspace in a file-scope device array
// instead of the handle's hipMalloc'd workspace.
#include <mutex>

#include "host.hpp"

using namespace phx;

namespace {

// 256 MiB per device, held from the first use of the library on a device until
// the process ends; the last 256 bytes hold the finiteness-scan flag word.
constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr size_t kFlagBytes = 256;

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

// Swaps the static scratch in as the handle's workspace for one call.
struct FixedWorkspace {
    Handle* h;
    char* ws;
    size_t cap, budget;
    bool timing;
    int32_t* dflag;
    explicit FixedWorkspace(Handle* h_)
        : h(h_), ws(h_->ws), cap(h_->ws_cap), budget(h_->budget), timing(h_->timing),
          dflag(h_->dflag) {
        h->ws = h->scratch;
        h->ws_cap = kScratchBytes - kFlagBytes;
        h->budget = kScratchBytes - kFlagBytes;
        h->timing = false;  // timing brackets create events
        h->dflag = reinterpret_cast<int32_t*>(h->scratch + kScratchBytes - kFlagBytes);
        h->fixed_ws = true;
    }
    ~FixedWorkspace() {
        h->ws = ws;
        h->ws_cap = cap;
        h->budget = budget;
        h->timing = timing;
        h->dflag = dflag;
        h->fixed_ws = false;
    }
};

}  // namespace

namespace phx {

hipError_t noalloc_scratch_init(int device, char** ptr) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[device] = static_cast<char*>(p);
    }
    *ptr = g_ptr[device];
    return hipSuccess;
}

}  // namespace phx

extern "C" {

phoebe_status phoebe_gpu_scatter_rates_noalloc(void* handle, const phoebe_system* sys,
                                               const int32_t k_mesh[3], const int32_t q_mesh[3],
                                               const int32_t* k_idx, int64_t nk,
                                               const int64_t* q_off, const int32_t* q_idx,
                                               const double* q_w, const phoebe_rate_params* par,
                                               phoebe_precision prec, double* gamma_out,
                                               uint8_t* band_mask, int32_t* kept_k_out,
                                               int64_t* n_kept_out, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    if (!h->scratch) {
        h->err = "the static scratch of this device could not be resolved";
        return PHOEBE_E_DEVICE;
    }
    FixedWorkspace fw(h);
    return phoebe_gpu_scatter_rates(handle, sys, k_mesh, q_mesh, k_idx, nk, q_off, q_idx, q_w, par,
                                    prec, gamma_out, band_mask, kept_k_out, n_kept_out, stream);
}

size_t phoebe_gpu_noalloc_scratch_bytes(void) { return kScratchBytes - kFlagBytes; }

}  // extern "C"
