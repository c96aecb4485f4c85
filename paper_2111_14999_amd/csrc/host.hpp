// Host-side helpers shared by the C ABI translation units: handle, workspace
// arena, error reporting, timing brackets, band-structure orchestration.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "ext.hpp"
#include "kernels.hpp"
#include "lowp.hpp"

namespace phx {

extern std::string g_create_error;

// Device address of the non-allocating entry point's static scratch on `device`
// (the current device), resolved once per device; hipSuccess or the lookup's error.
hipError_t noalloc_scratch_init(int device, char** ptr);



struct TimedLaunch {
    std::string name;
    hipEvent_t start, stop;
    double bytes = 0.0;  // algorithmic HBM bytes of the launch, where the host knows them
    // plus bytes_per_count[i] times counts the device leaves in dcount[i]
    const uint32_t* dcount[2] = {nullptr, nullptr};
    double bytes_per_count[2] = {0.0, 0.0};
};

struct KernelStat {
    std::string name;
    int64_t launches = 0;
    double total_ms = 0.0;
    double bytes = 0.0;
};

// Band and phonon tables of the last (system, mesh) the rate path built, kept
// while the table cache is on (phoebe_gpu_set_table_cache).
struct TableCache {
    bool valid = false;
    const void *h_r = nullptr, *phi_r = nullptr, *mass = nullptr;
    std::vector<int32_t> rh, rd;
    int nW = 0, nat = 0, n0 = 0, n1 = 0, n2 = 0;
    double omega_min = 0.0, kT = 0.0;
    char* mem = nullptr;
    size_t bytes = 0;
};

// Band and phonon tables of the system of the current rate call, built by a
// batched plan (same routines, same omega_min and kT) and lent to the plain calls
// it makes on replay; the rate path reads them in place of building its own.
struct PresetTables {
    double* eps;    // [N, nW]
    cd* U;          // [N, band, orbital] (transposed eigenvectors)
    double* omega;  // [N, nModes]
    cd* E;          // [N, nModes, nModes]
    double* nb;     // [N, nModes]
};

struct Handle {
    int device = 0;
    size_t budget = 0;
    char* ws = nullptr;
    size_t ws_cap = 0;
    std::string err;
    bool timing = false;
    int mesh_sum = 0;  // PHOEBE_MESH_SUM_AUTO / _DIRECT / _FACTORED
    bool check_finite = false;
    int32_t* dflag = nullptr;  // one device word for the finiteness scan (allocated on first use)
    char* scratch = nullptr;   // the device's static scratch of the non-allocating entry point
    bool fixed_ws = false;     // during such a call: ws is that scratch and is never reallocated
    bool table_cache = false;  // reuse band and phonon tables across rate calls
    int64_t inject_at = 0;     // testing: report the n-th successful HIP check as failed
    TableCache tc;
    const PresetTables* preset = nullptr;  // set only for the duration of a plan's plain call
    std::vector<TimedLaunch> pending;
    std::vector<KernelStat> stats;
};

struct Fail {
    phoebe_status st;
};

// Bump allocation over the handle's workspace.  A first pass with base ==
// nullptr only sizes the request.  A take beyond the capacity of a real pass
// (a sizing mistake) fails the call instead of handing out memory past the end.
struct Arena {
    char* base;
    size_t used = 0;
    size_t cap = SIZE_MAX;
    explicit Arena(char* b, size_t c = SIZE_MAX) : base(b), cap(c) {}
    template <class T>
    T* take(size_t count) {
        used = (used + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
        used += count * sizeof(T);
        if (base && used > cap) throw Fail{PHOEBE_E_NOMEM};
        return p;
    }
};

inline void set_err(Handle* h, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
inline void set_err(Handle* h, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->err = buf;
}

#define REQUIRE(h, cond, ...)                    \
    do {                                         \
        if (!(cond)) {                           \
            set_err((h), __VA_ARGS__);           \
            throw Fail{PHOEBE_E_INVALID};        \
        }                                        \
    } while (0)

// A failed HIP call ends the entry point with PHOEBE_E_DEVICE.  With fault
// injection armed (phoebe_gpu_set_fault_injection) the n-th successful check is
// reported as failed instead, after the device has finished the work in flight.
#define HIPCHK(h, expr)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        bool inj_ = false;                                                                \
        if (e_ == hipSuccess && (h)->inject_at > 0 && --(h)->inject_at == 0) {            \
            (void)hipDeviceSynchronize();                                                 \
            e_ = hipErrorUnknown;                                                         \
            inj_ = true;                                                                  \
        }                                                                                 \
        if (e_ != hipSuccess) {                                                           \
            set_err((h), "HIP error %s at %s:%d%s", hipGetErrorString(e_), __FILE__, __LINE__, \
                    inj_ ? " (injected)" : "");                                           \
            throw Fail{PHOEBE_E_DEVICE};                                                  \
        }                                                                                 \
    } while (0)

inline void ensure_ws(Handle* h, size_t bytes) {
    if (bytes <= h->ws_cap) return;
    if (h->fixed_ws) {
        set_err(h, "workspace of %zu bytes exceeds the %zu-byte static scratch of the "
                   "non-allocating entry point", bytes, h->ws_cap);
        throw Fail{PHOEBE_E_NOMEM};
    }
    if (bytes > h->budget) {
        set_err(h, "workspace of %zu bytes exceeds the budget of %zu bytes", bytes, h->budget);
        throw Fail{PHOEBE_E_NOMEM};
    }
    if (h->ws) {
        HIPCHK(h, hipDeviceSynchronize());
        char* old = h->ws;  // forgotten before the free is checked: never reused
        h->ws = nullptr;
        h->ws_cap = 0;
        HIPCHK(h, hipFree(old));
    }
    hipError_t e = hipMalloc(&h->ws, bytes);
    if (e != hipSuccess) {
        h->ws = nullptr;
        set_err(h, "hipMalloc of %zu workspace bytes failed: %s", bytes, hipGetErrorString(e));
        throw Fail{PHOEBE_E_NOMEM};
    }
    h->ws_cap = bytes;
}

// Timing brackets on the launch stream.
struct Timer {
    Handle* h;
    hipStream_t s;
    TimedLaunch t;
    bool on;
    Timer(Handle* h_, hipStream_t s_, const char* name) : h(h_), s(s_), on(h_->timing) {
        if (!on) return;
        t.name = name;
        HIPCHK(h, hipEventCreate(&t.start));
        HIPCHK(h, hipEventCreate(&t.stop));
        HIPCHK(h, hipEventRecord(t.start, s));
    }
    void done(double bytes = 0.0, const uint32_t* dcount = nullptr, double bytes_per_count = 0.0,
              const uint32_t* dcount2 = nullptr, double bytes_per_count2 = 0.0) {
        if (!on) return;
        t.bytes = bytes;
        t.dcount[0] = dcount;
        t.bytes_per_count[0] = bytes_per_count;
        t.dcount[1] = dcount2;
        t.bytes_per_count[1] = bytes_per_count2;
        HIPCHK(h, hipEventRecord(t.stop, s));
        h->pending.push_back(t);
        on = false;
    }
};

inline void flush_timing(Handle* h, hipStream_t s) {
    if (h->pending.empty()) return;
    HIPCHK(h, hipStreamSynchronize(s));
    for (auto& t : h->pending) {
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, t.start, t.stop));
        KernelStat* ks = nullptr;
        for (auto& k : h->stats)
            if (k.name == t.name) ks = &k;
        if (!ks) {
            h->stats.push_back(KernelStat{t.name, 0, 0.0, 0.0});
            ks = &h->stats.back();
        }
        ks->launches += 1;
        ks->total_ms += ms;
        ks->bytes += t.bytes;
        for (int i = 0; i < 2; ++i)
            if (t.dcount[i]) {
                uint32_t n = 0;
                HIPCHK(h, hipMemcpy(&n, t.dcount[i], sizeof(n), hipMemcpyDeviceToHost));
                ks->bytes += t.bytes_per_count[i] * n;
            }
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    h->pending.clear();
}

inline void check_system(Handle* h, const phoebe_system* sys, bool need_h, bool need_ph, bool need_g) {
    REQUIRE(h, sys != nullptr, "system is NULL");
    REQUIRE(h, sys->n_wannier >= 1, "n_wannier must be >= 1 (got %d)", sys->n_wannier);
    REQUIRE(h, sys->n_atoms >= 1, "n_atoms must be >= 1 (got %d)", sys->n_atoms);
    if (need_h) {
        REQUIRE(h, sys->n_rh >= 1 && sys->rh && sys->h_r, "H(R) arrays missing");
    }
    if (need_ph) {
        REQUIRE(h, sys->n_rd >= 1 && sys->rd && sys->phi_r && sys->mass, "force constants missing");
    }
    if (need_g) {
        REQUIRE(h, sys->n_re >= 1 && sys->re && sys->n_rp >= 1 && sys->rp && sys->g_rr,
                "g(Re,Rp) arrays missing");
    }
}

inline int32_t* upload_r(Handle* h, Arena& ar, const int32_t* host, int n, hipStream_t s) {
    int32_t* d = ar.take<int32_t>((size_t)3 * n);
    if (d) HIPCHK(h, hipMemcpyAsync(d, host, sizeof(int32_t) * 3 * n, hipMemcpyHostToDevice, s));
    return d;
}

inline int rmax_of(const int32_t* r, int n) {
    int m = 0;
    for (int i = 0; i < 3 * n; ++i) m = std::max(m, std::abs(r[i]));
    return m;
}

// ---------------------------------------------------------------------------
// band structure on a set of points (fractional coordinates or mesh indices)
// ---------------------------------------------------------------------------
struct BandBufs {
    double* eps;
    cd* U;
};

inline void electron_bands_dev(Handle* h, Arena& ar, const phoebe_system* sys, const int32_t* rh_d,
                        const double* frac, const int32_t* idx, Mesh m, int64_t np, double* eps,
                        cd* U, hipStream_t s) {
    const int nW = sys->n_wannier, nR = sys->n_rh;
    cd* P = ar.take<cd>((size_t)np * nR);
    cd* H = ar.take<cd>((size_t)np * nW * nW);
    if (!ar.base) return;
    HIPCHK(h, launch_phase_table(frac, idx, m, np, rh_d, nR, P, nR, s));
    Timer t(h, s, "bands_fft");
    HIPCHK(h, launch_zgemm(P, nR, reinterpret_cast<const cd*>(sys->h_r), (int64_t)nW * nW, H,
                           (int64_t)nW * nW, np, (int64_t)nW * nW, nR, s));
    t.done();
    Timer te(h, s, "eig_jacobi");
    HIPCHK(h, launch_eig_herm(H, nW, np, eps, U, s));
    te.done();
}

inline void phonon_dev(Handle* h, Arena& ar, const phoebe_system* sys, const int32_t* rd_d,
                const double* frac, const int32_t* idx, Mesh m, int64_t np, double omega_min,
                double kT, double* omega, cd* E, double* nb, cd* z_out, hipStream_t s) {
    const int nm = 3 * sys->n_atoms, nR = sys->n_rd;
    cd* P = ar.take<cd>((size_t)np * nR);
    cd* phic = ar.take<cd>((size_t)nR * nm * nm);
    cd* D = ar.take<cd>((size_t)np * nm * nm);
    double* lam = ar.take<double>((size_t)np * nm);
    cd* z = z_out ? z_out : ar.take<cd>((size_t)np * nm * nm);
    if (!ar.base) return;
    HIPCHK(h, launch_phase_table(frac, idx, m, np, rd_d, nR, P, nR, s));
    HIPCHK(h, launch_mass_weight(sys->phi_r, sys->mass, nR, nm, phic, s));
    HIPCHK(h, launch_zgemm(P, nR, phic, (int64_t)nm * nm, D, (int64_t)nm * nm, np,
                           (int64_t)nm * nm, nR, s));
    HIPCHK(h, launch_eig_herm(D, nm, np, lam, z, s));
    HIPCHK(h, launch_phonon_post(lam, z, sys->mass, sys->n_atoms, np, omega_min, kT, omega, E, nb,
                                 s));
}

inline void check_polar(Handle* h, const phoebe_system* sys) {
    const phoebe_polar* p = sys->polar;
    REQUIRE(h, p->born != nullptr, "polar: Born charges are NULL");
    REQUIRE(h, std::isfinite(p->alpha) && p->alpha > 0.0, "polar: alpha must be > 0");
    REQUIRE(h, p->g_max >= 0 && p->g_max <= 8, "polar: g_max must be in [0, 8]");
    REQUIRE(h, sys->n_atoms <= 10, "polar: at most 10 atoms");
    for (int i = 0; i < 9; ++i) REQUIRE(h, std::isfinite(p->eps_inf[i]), "polar: eps_inf not finite");
    for (int i = 0; i < 9 * sys->n_atoms; ++i)
        REQUIRE(h, std::isfinite(p->born[i]), "polar: Born charges not finite");
}

inline PolarDev polar_dev(const phoebe_system* sys, const double* born_dev) {
    PolarDev d{};
    d.born = born_dev;
    for (int i = 0; i < 9; ++i) d.eps[i] = sys->polar->eps_inf[i];
    d.alpha = sys->polar->alpha;
    d.g_max = sys->polar->g_max;
    d.nat = sys->n_atoms;
    return d;
}

// Group velocities at points (fractional or mesh): the phase table, its
// k-derivative form, dH/dk_a on MFMA and the projection with the eigenvectors
// U (u_transposed: U[p, band, orbital], else columns).
inline void velocity_dev(Handle* h, Arena& ar, const phoebe_system* sys, const int32_t* rh_d,
                         const double* frac, Mesh m, int64_t np, const double* eps, const cd* U,
                         bool u_transposed, double* v, int32_t* bad, hipStream_t s) {
    const int nW = sys->n_wannier, nR = sys->n_rh;
    cd* P = ar.take<cd>((size_t)np * nR);
    cd* Pv = ar.take<cd>((size_t)np * 3 * nR);
    cd* dH = ar.take<cd>((size_t)np * 3 * nW * nW);
    if (!ar.base) return;
    HIPCHK(h, launch_phase_table(frac, nullptr, m, np, rh_d, nR, P, nR, s));
    HIPCHK(h, launch_velocity_phases(P, np, rh_d, nR, Pv, s));
    HIPCHK(h, launch_zgemm(Pv, nR, reinterpret_cast<const cd*>(sys->h_r), (int64_t)nW * nW, dH,
                           (int64_t)nW * nW, np * 3, (int64_t)nW * nW, nR, s));
    HIPCHK(h, launch_zero(bad, sizeof(int32_t), s));
    HIPCHK(h, launch_group_velocities(dH, U, u_transposed, eps, np, nW, 1e-6, v, bad, s));
}

// Optional finiteness scan of a system's tensors (phoebe_gpu_set_check_finite).
inline void scan_finite(Handle* h, const phoebe_system* sys, bool hh, bool ph, bool g,
                        hipStream_t s) {
    if (!h->check_finite) return;
    if (!h->dflag && h->fixed_ws) {
        set_err(h, "no flag word for the finiteness scan");
        throw Fail{PHOEBE_E_DEVICE};
    }
    if (!h->dflag) {
        int32_t* p = nullptr;
        const hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), sizeof(int32_t));
        if (e == hipSuccess) h->dflag = p;  // kept (and freed with the handle) once allocated
        HIPCHK(h, e);
    }
    int32_t* flag = h->dflag;
    int32_t bad = 0;
    {
        HIPCHK(h, launch_zero(flag, sizeof(int32_t), s));
        const int nW = sys->n_wannier, nm = 3 * sys->n_atoms;
        if (hh) HIPCHK(h, launch_nonfinite(reinterpret_cast<const double*>(sys->h_r),
                                           (int64_t)sys->n_rh * nW * nW * 2, flag, s));
        if (ph) {
            HIPCHK(h, launch_nonfinite(sys->phi_r, (int64_t)sys->n_rd * nm * nm, flag, s));
            HIPCHK(h, launch_nonfinite(sys->mass, sys->n_atoms, flag, s));
        }
        if (g) HIPCHK(h, launch_nonfinite(reinterpret_cast<const double*>(sys->g_rr),
                                          (int64_t)sys->n_re * sys->n_rp * nm * nW * nW * 2, flag, s));
        HIPCHK(h, hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
    }
    if (bad) {
        set_err(h, "an input tensor holds NaN or infinity");
        throw Fail{PHOEBE_E_NUMERIC};
    }
}

// Marks the entry point as a named range for tracing tools (rocprofv3 --marker-trace).
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
};

inline phoebe_status run(Handle* h, const char* name, const std::function<void()>& body) {
    TraceRange range(name);
    try {
        h->err.clear();
        body();
        return PHOEBE_OK;
    } catch (const Fail& f) {
        if (h->err.empty()) h->err = "workspace sizing error (internal)";
        return f.st;
    } catch (const std::bad_alloc&) {
        set_err(h, "host allocation failed");
        return PHOEBE_E_NOMEM;
    }
}


}  // namespace phx
