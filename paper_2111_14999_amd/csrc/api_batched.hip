// C ABI of the batched form: many independent systems, band tables and windows
// built once per plan, then one captured hipGraph whose core is the persistent
// multi-system rate kernel (FP32 contractions, FP64 tables and rates), one
// launch per tile shape in use, each draining the queue of its shape's tasks.  Tile
// shapes per system come from an autotuner that times the candidates and can
// keep its choices in a small JSON cache file.
#include <chrono>
#include <fstream>
#include <map>
#include <sstream>

#include "batched.hpp"
#include "host.hpp"

using namespace phx;

namespace {

struct SysPlan {
    // per-system device data (inside the plan's allocation)
    int32_t *rh, *rd, *re, *rp, *rp_packed;
    double *eps, *focc, *omega, *nb, *bmin, *bmax, *wmax;
    cd *U, *E;
    uint8_t* mask;
    int32_t *flag, *kept, *cnt, *rowflag, *ids;
    int32_t *st_row, *st_band, *st_kmesh, *st_mlo, *st_mhi;
    cd* P1;              // [rows, n_re] phases of the kept k
    cf* F;               // [states, rp_pad, nc_pad]
    double* partial;     // [states, n_qtiles]
    double* gamma;       // [rows, nW]
    // sizes
    Mesh mesh;
    int64_t N = 0, rows = 0;
    int states = 0;
    int nW = 0, nm = 0, n_re = 0, n_rp = 0, rmax = 0, rp_pad = 0;
    int tq = 2, tn = 1, nc_pad = 64, n_qtiles = 0;
    int stage = 0;  // the tile stages its rotation operands in LDS (chosen per tile shape)
    double sigma = 0.0;
    std::vector<int32_t> strow;
    const phoebe_system* sys = nullptr;
    // a full-mesh system of at most 16 Wannier functions runs as one plain rate call
    // (the factorised mesh sums) when the plan is replayed, not in the graph
    bool plain = false;
    phoebe_rate_params par{};
    // the plan's own copy of the system (its lattice lists on the host), so that a
    // replay does not read the caller's structs after the plan call returned
    phoebe_system sys_copy{};
    std::vector<int32_t> rh_v, rd_v, re_v, rp_v;
};

// the persistent kernel of the graph takes this system's states
bool in_graph(const SysPlan& p) { return p.states > 0 && !p.plain; }

struct Plan {
    Handle* h = nullptr;
    int n_sys = 0;
    char* mem = nullptr;
    size_t mem_bytes = 0;
    std::vector<SysPlan> sp;
    SysDesc* d_desc = nullptr;
    BTask* d_tasks = nullptr;
    int* d_head = nullptr;
    cf* G = nullptr;
    int n_tasks = 0;
    // tasks, dynamic LDS and work-groups of each shape's persistent kernel; the
    // task list holds the shapes' queues one after the other
    int n_tasks_shape[kBatchedShapes] = {};
    size_t lds_shape[kBatchedShapes] = {};
    int n_wg_shape[kBatchedShapes] = {};
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double tune_ms = 0.0;
};

constexpr int kBK = 64;  // kept k per stage-1 batch

int nc_pad_for(int nc, int tn) {
    const int w = 64 * tn;
    return (nc + w - 1) / w * w;
}

std::string tune_key(const SysPlan& p) {
    std::ostringstream o;
    o << "nm=" << p.nm << ",nW=" << p.nW << ",nrp=" << p.n_rp << ",rmax=" << p.rmax
      << ",nq=" << p.N;
    return o.str();
}

// cache file: one entry per line, {"key": "...", "tq": T, "tn": T, "us_per_task": X}
std::map<std::string, std::pair<int, int>> load_cache(const char* path) {
    std::map<std::string, std::pair<int, int>> m;
    if (!path) return m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t k0 = line.find("\"key\": \"");
        if (k0 == std::string::npos) continue;
        const size_t k1 = line.find('"', k0 + 8);
        const size_t a = line.find("\"tq\": ");
        const size_t b = line.find("\"tn\": ");
        if (k1 == std::string::npos || a == std::string::npos || b == std::string::npos) continue;
        m[line.substr(k0 + 8, k1 - k0 - 8)] = {std::atoi(line.c_str() + a + 6),
                                              std::atoi(line.c_str() + b + 6)};
    }
    return m;
}

void save_cache(const char* path, const std::map<std::string, std::pair<int, int>>& m,
                const std::map<std::string, double>& us) {
    if (!path) return;
    std::ofstream f(path);
    f << "{\"entries\": [\n";
    size_t i = 0;
    for (auto& kv : m) {
        auto it = us.find(kv.first);
        f << "{\"key\": \"" << kv.first << "\", \"tq\": " << kv.second.first
          << ", \"tn\": " << kv.second.second << ", \"us_per_task\": "
          << (it == us.end() ? 0.0 : it->second) << "}" << (++i < m.size() ? "," : "") << "\n";
    }
    f << "]}\n";
}

// smallest TN whose 64*TN columns hold the system's nModes*nW in one pass
int tn_for(int nc) {
    static const int tns[] = {1, 2, 3, 4, 6, 8, 12, 16};
    for (int tn : tns)
        if (64 * tn >= nc) return tn;
    return 0;
}

void fill_desc(const SysPlan& p, SysDesc& d) {
    RateArgsLP& a = d.a;
    a = RateArgsLP{};
    a.F = p.F;
    a.rp_pad = p.rp_pad;
    a.nc_pad = p.nc_pad;
    a.n_rp = p.n_rp;
    a.rp_packed = p.rp_packed;
    a.rmax = p.rmax;
    a.mesh = p.mesh;
    a.nq_mesh = p.N;
    a.st_kmesh = p.st_kmesh;
    a.st_band = p.st_band;
    a.st_row = p.st_row;
    a.st_mlo = p.st_mlo;
    a.st_mhi = p.st_mhi;
    a.eps = p.eps;
    a.focc = p.focc;
    a.U = p.U;
    a.omega = p.omega;
    a.nb = p.nb;
    a.E = p.E;
    a.nW = p.nW;
    a.nm = p.nm;
    a.sigma = p.sigma;
    a.partial = p.partial;
    a.n_qtiles = p.n_qtiles;
    a.stage = p.stage;
    d.tq = p.tq;
    d.tn = p.tn;
}

// work-groups of a persistent launch: as many per CU as the LDS of its largest
// tile allows, at most 8 (those beyond what the registers allow start when
// others end; a queue task never waits on another)
int persistent_wgs(size_t lds) {
    return 256 * std::max(1, std::min(8, (int)((160 * 1024) / std::max<size_t>(lds, 1))));
}

// stage 1 + fold of states [s0, s1) of one system into F (rows of those states)
void enqueue_stage1(Handle* h, const SysPlan& p, cf* G, int s0, int s1, cf* F, int nc_pad,
                    hipStream_t s) {
    const int64_t NC2 = (int64_t)p.n_rp * p.nm * p.nW * p.nW;
    int a = s0;
    while (a < s1) {
        const int64_t r0 = p.strow[a];
        int b = a;
        while (b < s1 && p.strow[b] < r0 + kBK) ++b;
        const int64_t nb = std::min<int64_t>(kBK, p.rows - r0);
        HIPCHK(h, launch_cgemm_lp(PHOEBE_FP32, p.P1 + r0 * p.n_re, p.n_re,
                                  reinterpret_cast<const cd*>(p.sys->g_rr), NC2, G, NC2, nb, NC2,
                                  p.n_re, s));
        HIPCHK(h, launch_fold_uk_lp(PHOEBE_FP32, G, NC2, p.U, p.st_row + a, (int)r0,
                                    p.st_kmesh + a, p.st_band + a, b - a, p.n_rp, p.nm, p.nW,
                                    p.nW, p.rp_pad, nc_pad, F + (int64_t)(a - s0) * p.rp_pad * nc_pad,
                                    s));
        a = b;
    }
}

void destroy_plan(Plan* P) {
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->cs) (void)hipStreamDestroy(P->cs);
    if (P->mem) (void)hipFree(P->mem);
    delete P;
}

}  // namespace

extern "C" {

phoebe_status phoebe_gpu_batched_plan(void* handle, const phoebe_system* systems, int32_t n_sys,
                                      const int32_t* meshes, const phoebe_rate_params* params,
                                      phoebe_precision prec, const char* tune_cache, void** plan_out,
                                      int64_t* n_kept_out, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Plan* P = nullptr;
    const phoebe_status st = run(h, __func__, [&] {
        REQUIRE(h, plan_out != nullptr, "plan out-pointer is NULL");
        *plan_out = nullptr;
        REQUIRE(h, systems && meshes && params && n_sys >= 1, "systems/meshes/params missing");
        if (prec != PHOEBE_FP32) {
            set_err(h, "the batched form runs complex64 (PHOEBE_FP32) contractions");
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        HIPCHK(h, hipSetDevice(h->device));
        P = new Plan();
        P->h = h;
        P->n_sys = n_sys;
        P->sp.resize(n_sys);
        for (int i = 0; i < n_sys; ++i) {
            const phoebe_system* sys = &systems[i];
            check_system(h, sys, true, true, true);
            const phoebe_rate_params* par = &params[i];
            if (sys->polar || par->smearing != PHOEBE_SMEAR_GAUSSIAN) {
                set_err(h, "system %d: the batched form takes non-polar systems with a fixed width", i);
                throw Fail{PHOEBE_E_UNSUPPORTED};
            }
            REQUIRE(h, std::isfinite(par->sigma) && par->sigma > 0.0, "system %d: sigma must be > 0", i);
            REQUIRE(h, std::isfinite(par->kT) && par->kT > 0.0, "system %d: kT must be > 0", i);
            REQUIRE(h, std::isfinite(par->omega_min) && par->omega_min >= 0.0, "system %d: omega_min", i);
            REQUIRE(h, meshes[3 * i] >= 1 && meshes[3 * i + 1] >= 1 && meshes[3 * i + 2] >= 1,
                    "system %d: mesh must be >= 1", i);
            SysPlan& p = P->sp[i];
            p.sys_copy = *sys;
            p.rh_v.assign(sys->rh, sys->rh + 3 * (size_t)sys->n_rh);
            p.rd_v.assign(sys->rd, sys->rd + 3 * (size_t)sys->n_rd);
            p.re_v.assign(sys->re, sys->re + 3 * (size_t)sys->n_re);
            p.rp_v.assign(sys->rp, sys->rp + 3 * (size_t)sys->n_rp);
            p.sys_copy.rh = p.rh_v.data();
            p.sys_copy.rd = p.rd_v.data();
            p.sys_copy.re = p.re_v.data();
            p.sys_copy.rp = p.rp_v.data();
            p.sys = &p.sys_copy;
            p.par = *par;
            p.mesh = Mesh{meshes[3 * i], meshes[3 * i + 1], meshes[3 * i + 2]};
            p.N = (int64_t)p.mesh.n0 * p.mesh.n1 * p.mesh.n2;
            REQUIRE(h, p.N <= (int64_t)1 << 26, "system %d: mesh too large", i);
            p.nW = sys->n_wannier;
            p.nm = 3 * sys->n_atoms;
            if (p.nW > 32 || p.nm > 32) {
                set_err(h, "system %d: nW > 32 or nModes > 32 is not supported", i);
                throw Fail{PHOEBE_E_UNSUPPORTED};
            }
            p.n_re = sys->n_re;
            p.n_rp = sys->n_rp;
            p.rmax = rmax_of(sys->rp, sys->n_rp);
            REQUIRE(h, p.rmax <= 100, "system %d: |Rp| components above 100", i);
            p.rp_pad = (p.n_rp + 3) & ~3;
            p.sigma = par->sigma;
        }

        // ---- per-system tables, windows and state lists ----
        // plan memory, part 1: tables and state lists (sized before anything runs)
        auto carve_tables = [&](Arena& ar, SysPlan& p) {
            p.rh = ar.take<int32_t>(3 * (size_t)p.sys->n_rh);
            p.rd = ar.take<int32_t>(3 * (size_t)p.sys->n_rd);
            p.re = ar.take<int32_t>(3 * (size_t)p.n_re);
            p.rp = ar.take<int32_t>(3 * (size_t)p.n_rp);
            p.rp_packed = ar.take<int32_t>(p.n_rp);
            p.eps = ar.take<double>((size_t)p.N * p.nW);
            p.focc = ar.take<double>((size_t)p.N * p.nW);
            p.U = ar.take<cd>((size_t)p.N * p.nW * p.nW);
            p.omega = ar.take<double>((size_t)p.N * p.nm);
            p.nb = ar.take<double>((size_t)p.N * p.nm);
            p.E = ar.take<cd>((size_t)p.N * p.nm * p.nm);
            p.bmin = ar.take<double>(p.nW);
            p.bmax = ar.take<double>(p.nW);
            p.wmax = ar.take<double>(1);
            p.mask = ar.take<uint8_t>((size_t)p.N * p.nW);
            p.flag = ar.take<int32_t>(p.N);
            p.kept = ar.take<int32_t>(p.N);
            p.cnt = ar.take<int32_t>(2);
            p.rowflag = ar.take<int32_t>((size_t)p.N * p.nW);
            p.ids = ar.take<int32_t>((size_t)p.N * p.nW);
            p.st_row = ar.take<int32_t>((size_t)p.N * p.nW);
            p.st_band = ar.take<int32_t>((size_t)p.N * p.nW);
            p.st_kmesh = ar.take<int32_t>((size_t)p.N * p.nW);
            p.st_mlo = ar.take<int32_t>((size_t)p.N * p.nW);
            p.st_mhi = ar.take<int32_t>((size_t)p.N * p.nW);
            p.P1 = ar.take<cd>((size_t)p.N * p.n_re);
            p.gamma = ar.take<double>((size_t)p.N * p.nW);
        };
        size_t tables_bytes = 0;
        {
            Arena dry(nullptr);
            for (auto& p : P->sp) carve_tables(dry, p);
            tables_bytes = (dry.used + 4096 + 255) & ~(size_t)255;  // part 2 starts aligned
        }
        // band scratch comes from the handle workspace, one system at a time
        size_t scratch = 0;
        for (auto& p : P->sp) {
            Arena d1(nullptr), d2(nullptr);
            electron_bands_dev(h, d1, p.sys, nullptr, nullptr, nullptr, p.mesh, p.N, nullptr,
                               nullptr, s);
            phonon_dev(h, d2, p.sys, nullptr, nullptr, nullptr, p.mesh, p.N, 0, 0, nullptr,
                       nullptr, nullptr, nullptr, s);
            scratch = std::max(scratch, std::max(d1.used, d2.used));
        }
        ensure_ws(h, scratch + 256);
        if (tables_bytes > h->budget) {
            set_err(h, "batched tables need %zu bytes, over the budget", tables_bytes);
            throw Fail{PHOEBE_E_NOMEM};
        }
        char* tables_mem = nullptr;
        if (hipMalloc(&tables_mem, tables_bytes) != hipSuccess) {
            set_err(h, "hipMalloc of %zu bytes for the batched tables failed", tables_bytes);
            throw Fail{PHOEBE_E_NOMEM};
        }
        P->mem = tables_mem;
        P->mem_bytes = tables_bytes;
        Arena tar(tables_mem, tables_bytes);
        for (int i = 0; i < n_sys; ++i) {
            SysPlan& p = P->sp[i];
            const phoebe_rate_params* par = &params[i];
            carve_tables(tar, p);
            const phoebe_system* sys = p.sys;
            HIPCHK(h, hipMemcpyAsync(p.rh, sys->rh, 12 * (size_t)sys->n_rh, hipMemcpyHostToDevice, s));
            HIPCHK(h, hipMemcpyAsync(p.rd, sys->rd, 12 * (size_t)sys->n_rd, hipMemcpyHostToDevice, s));
            HIPCHK(h, hipMemcpyAsync(p.re, sys->re, 12 * (size_t)p.n_re, hipMemcpyHostToDevice, s));
            HIPCHK(h, hipMemcpyAsync(p.rp, sys->rp, 12 * (size_t)p.n_rp, hipMemcpyHostToDevice, s));
            std::vector<int32_t> packed(p.n_rp);
            for (int r = 0; r < p.n_rp; ++r)
                packed[r] = (sys->rp[3 * r] + p.rmax) | ((sys->rp[3 * r + 1] + p.rmax) << 8) |
                            ((sys->rp[3 * r + 2] + p.rmax) << 16);
            HIPCHK(h, hipMemcpyAsync(p.rp_packed, packed.data(), 4 * (size_t)p.n_rp,
                                     hipMemcpyHostToDevice, s));
            HIPCHK(h, hipStreamSynchronize(s));
            {
                Arena b1(h->ws, h->ws_cap), b2(h->ws, h->ws_cap);
                electron_bands_dev(h, b1, sys, p.rh, nullptr, nullptr, p.mesh, p.N, p.eps, p.U, s);
                // the rate kernels read each eigenvector contiguously
                HIPCHK(h, launch_transpose_batch(p.U, p.N, p.nW, s));
                phonon_dev(h, b2, sys, p.rd, nullptr, nullptr, p.mesh, p.N, par->omega_min, par->kT,
                           p.omega, p.E, p.nb, nullptr, s);
            }
            HIPCHK(h, launch_fermi(p.eps, p.N * p.nW, par->mu, par->kT, p.focc, s));
            HIPCHK(h, launch_band_extrema(p.eps, p.N, p.nW, p.omega, p.N, p.nm, p.bmin, p.bmax,
                                          p.wmax, s));
            HIPCHK(h, launch_window(p.eps, p.N, p.nW, par->win_lo, par->win_hi, p.mask, p.flag, s));
            HIPCHK(h, launch_compact(p.flag, p.N, p.kept, p.cnt, s));
            int32_t c = 0;
            HIPCHK(h, hipMemcpyAsync(&c, p.cnt, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            p.rows = c;
            if (n_kept_out) n_kept_out[i] = c;
            HIPCHK(h, launch_zero(p.gamma, (size_t)p.N * p.nW * sizeof(double), s));
            if (p.rows == 0) continue;
            HIPCHK(h, launch_gather_rows(p.mask, p.kept, p.rows, p.nW, p.rowflag, nullptr, nullptr, s));
            HIPCHK(h, launch_compact(p.rowflag, p.rows * p.nW, p.ids, p.cnt + 1, s));
            HIPCHK(h, hipMemcpyAsync(&c, p.cnt + 1, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            p.states = c;
            if (p.states == 0) continue;
            HIPCHK(h, launch_build_states(p.ids, p.states, p.nW, p.kept, p.eps, p.bmin, p.bmax,
                                          p.wmax, 27.5 * par->sigma, p.st_row, p.st_band, p.st_kmesh,
                                          p.st_mlo, p.st_mhi, s));
            HIPCHK(h, launch_phase_table(nullptr, p.kept, p.mesh, p.rows, p.re, p.n_re, p.P1, p.n_re, s));
            p.strow.resize(p.states);
            HIPCHK(h, hipMemcpyAsync(p.strow.data(), p.st_row, 4 * (size_t)p.states,
                                     hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            // where the plain rate call takes the factorised sums (its automatic rule: the
            // full mesh, nW <= 32, an Rp box at most 31 wide and half the Rp count), they
            // do tens of times fewer operations than the persistent kernel's direct
            // contraction, so the system runs as such a call
            const int wbox = 2 * p.rmax + 1;
            p.plain = h->mesh_sum != PHOEBE_MESH_SUM_DIRECT && line_rates_ncpad(p.nm, p.nW) > 0 &&
                      wbox <= 31 && 2 * wbox <= p.n_rp && p.mesh.n0 <= 1024 &&
                      (int64_t)p.mesh.n1 * p.mesh.n2 <= 65535 &&
                      line_rates_lds(wbox, p.mesh.n0, p.nm, true) <= 64 * 1024;
            if (p.plain) p.tq = p.tn = 0;
        }

        // ---- stage-1 buffer, autotuning of (TQ, TN) per system ----
        int64_t g_max = 0;
        for (auto& p : P->sp)
            if (in_graph(p)) g_max = std::max<int64_t>(g_max, (int64_t)kBK * p.n_rp * p.nm * p.nW * p.nW);
        const auto t_tune0 = std::chrono::steady_clock::now();
        auto cache = load_cache(tune_cache);
        std::map<std::string, double> cache_us;
        size_t tune_f = 0;
        for (auto& p : P->sp)
            tune_f = std::max(tune_f, (size_t)4 * p.rp_pad * 64 * std::max(1, tn_for(p.nm * p.nW)));
        {
            // workspace: G, F of the tuning states, partials, one descriptor, tasks, head
            const size_t need = (size_t)g_max * sizeof(cf) + tune_f * sizeof(cf) + 1024 * 1024 * 8;
            ensure_ws(h, std::max(need, scratch) + 4096);
        }
        for (auto& p : P->sp) {
            if (!in_graph(p)) continue;
            const std::string key = tune_key(p);
            auto it = cache.find(key);
            if (it != cache.end() &&
                batched_tile_supported(it->second.first, it->second.second, p.nm * p.nW) &&
                batched_lds(it->second.first, p.rmax, p.rp_pad, nc_pad_for(p.nm * p.nW, it->second.second), p.nm, p.nW, false) <= 150 * 1024) {
                p.tq = it->second.first;
                p.tn = it->second.second;
                continue;
            }
            const int ns = std::min(p.states, 4);
            double best = 1e300;
            int btq = 0, btn = 0;
            // the one-pass TN at both q-tile heights
            const int tn1 = tn_for(p.nm * p.nW);
            const int cands[2][2] = {{2, tn1}, {1, tn1}};
            for (auto& c : cands) {
                const int tq = c[0], tn = c[1];
                if (!batched_tile_supported(tq, tn, p.nm * p.nW)) continue;
                const int ncp = nc_pad_for(p.nm * p.nW, tn);
                const size_t lds0 = batched_lds(tq, p.rmax, p.rp_pad, ncp, p.nm, p.nW, false);
                const size_t lds1 = batched_lds(tq, p.rmax, p.rp_pad, ncp, p.nm, p.nW, true);
                if (lds0 > 150 * 1024) continue;
                const bool stg = batched_stage_pays(batched_shape(tq, tn), lds0, lds1);
                const size_t lds = stg ? lds1 : lds0;
                Arena wa(h->ws);
                cf* G = wa.take<cf>(g_max);
                cf* F = wa.take<cf>((size_t)ns * p.rp_pad * ncp);
                const int nqt = (int)((p.N + 16 * tq - 1) / (16 * tq));
                double* part = wa.take<double>((size_t)ns * nqt);
                SysDesc* dd = wa.take<SysDesc>(1);
                BTask* tk = wa.take<BTask>((size_t)ns * nqt);
                int* head = wa.take<int>(2);
                if (wa.used > h->ws_cap) continue;
                enqueue_stage1(h, p, G, 0, ns, F, ncp, s);
                SysPlan q = p;
                q.tq = tq;
                q.tn = tn;
                q.nc_pad = ncp;
                q.F = F;
                q.partial = part;
                q.n_qtiles = nqt;
                q.stage = stg ? 1 : 0;
                SysDesc d{};
                fill_desc(q, d);
                std::vector<BTask> tv;
                for (int a = 0; a < ns; ++a)
                    for (int t = 0; t < nqt; ++t) tv.push_back(BTask{0, a, t, 0});
                HIPCHK(h, hipMemcpyAsync(dd, &d, sizeof d, hipMemcpyHostToDevice, s));
                HIPCHK(h, hipMemcpyAsync(tk, tv.data(), sizeof(BTask) * tv.size(), hipMemcpyHostToDevice, s));
                double t_best = 1e300;
                for (int rep = 0; rep < 2; ++rep) {
                    hipEvent_t e0, e1;
                    HIPCHK(h, hipEventCreate(&e0));
                    HIPCHK(h, hipEventCreate(&e1));
                    HIPCHK(h, launch_zero(head, 8, s));
                    HIPCHK(h, hipEventRecord(e0, s));
                    HIPCHK(h, launch_batched_rates(batched_shape(tq, tn), dd, tk, (int)tv.size(),
                                                   head, persistent_wgs(lds), lds, s));
                    HIPCHK(h, hipEventRecord(e1, s));
                    HIPCHK(h, hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    t_best = std::min(t_best, (double)ms);
                }
                const double per_q = t_best / ((double)ns * (double)p.N);
                if (per_q < best) {
                    best = per_q;
                    btq = tq;
                    btn = tn;
                }
            }
            if (btq == 0) {
                set_err(h, "no tile shape of the batched kernel fits this system (nModes*nW = %d)",
                        p.nm * p.nW);
                throw Fail{PHOEBE_E_UNSUPPORTED};
            }
            p.tq = btq;
            p.tn = btn;
            cache[key] = {btq, btn};
            cache_us[key] = best * 1e3 * 16 * btq;  // microseconds per task
        }
        HIPCHK(h, hipStreamSynchronize(s));
        save_cache(tune_cache, cache, cache_us);
        P->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_tune0).count();

        // ---- plan memory, part 2: F, partials, descriptors, tasks ----
        std::vector<BTask> tasks;
        std::vector<int> order;
        for (int i = 0; i < n_sys; ++i)
            if (in_graph(P->sp[i])) order.push_back(i);
        // longest tasks first so the queue's tail holds the short ones
        std::sort(order.begin(), order.end(), [&](int a, int b) {
            const SysPlan &x = P->sp[a], &y = P->sp[b];
            return (double)x.n_rp * x.nm * x.nW * 16 * x.tq > (double)y.n_rp * y.nm * y.nW * 16 * y.tq;
        });
        Arena dry(nullptr);
        size_t f_total = 0, part_total = 0;
        // per shape: the largest LDS block of its systems, without and with staging;
        // staging is chosen for the whole shape (one kernel, one LDS size)
        size_t lds0[kBatchedShapes] = {}, lds1[kBatchedShapes] = {};
        for (auto& p : P->sp) {
            if (!in_graph(p)) continue;
            p.nc_pad = nc_pad_for(p.nm * p.nW, p.tn);
            p.n_qtiles = (int)((p.N + 16 * p.tq - 1) / (16 * p.tq));
            f_total += (size_t)p.states * p.rp_pad * p.nc_pad;
            part_total += (size_t)p.states * p.n_qtiles;
            const int sh = batched_shape(p.tq, p.tn);
            lds0[sh] = std::max(lds0[sh], batched_lds(p.tq, p.rmax, p.rp_pad, p.nc_pad, p.nm, p.nW, false));
            lds1[sh] = std::max(lds1[sh], batched_lds(p.tq, p.rmax, p.rp_pad, p.nc_pad, p.nm, p.nW, true));
        }
        for (int sh = 0; sh < kBatchedShapes; ++sh) {
            if (!lds0[sh]) continue;
            const bool stg = batched_stage_pays(sh, lds0[sh], lds1[sh]);
            P->lds_shape[sh] = stg ? lds1[sh] : lds0[sh];
            for (auto& p : P->sp)
                if (in_graph(p) && batched_shape(p.tq, p.tn) == sh) p.stage = stg ? 1 : 0;
        }
        for (int sh = 0; sh < kBatchedShapes; ++sh)
            for (int i : order) {
                const SysPlan& p = P->sp[i];
                if (batched_shape(p.tq, p.tn) != sh) continue;
                for (int a = 0; a < p.states; ++a)
                    for (int t = 0; t < p.n_qtiles; ++t) tasks.push_back(BTask{i, a, t, 0});
                P->n_tasks_shape[sh] += p.states * p.n_qtiles;
            }
        P->n_tasks = (int)tasks.size();
        // (each take below starts on a 256-byte boundary: two per graph system, four more)
        size_t n_takes = 4;
        for (auto& p : P->sp) n_takes += in_graph(p) ? 2 : 0;
        const size_t run_bytes = f_total * sizeof(cf) + part_total * sizeof(double) +
                                 (size_t)n_sys * sizeof(SysDesc) + tasks.size() * sizeof(BTask) +
                                 (size_t)g_max * sizeof(cf) + (n_takes + 1) * 256;
        if (P->mem_bytes + run_bytes > h->budget) {
            set_err(h, "batched plan needs %zu bytes, over the budget", P->mem_bytes + run_bytes);
            throw Fail{PHOEBE_E_NOMEM};
        }
        // grow the plan allocation: tables are copied to a new block that also holds part 2
        char* mem2 = nullptr;
        if (hipMalloc(&mem2, P->mem_bytes + run_bytes) != hipSuccess) {
            set_err(h, "hipMalloc of %zu bytes for the batched plan failed", P->mem_bytes + run_bytes);
            throw Fail{PHOEBE_E_NOMEM};
        }
        char* old = P->mem;  // the plan owns the new block from here on
        P->mem = mem2;
        HIPCHK(h, hipStreamSynchronize(s));
        HIPCHK(h, hipMemcpy(mem2, old, P->mem_bytes, hipMemcpyDeviceToDevice));
        const ptrdiff_t shift = mem2 - old;
        HIPCHK(h, hipFree(old));
        auto mv = [&](auto*& ptr) {
            if (ptr) ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(reinterpret_cast<char*>(ptr) + shift);
        };
        for (auto& p : P->sp) {
            mv(p.rh); mv(p.rd); mv(p.re); mv(p.rp); mv(p.rp_packed); mv(p.eps); mv(p.focc);
            mv(p.omega); mv(p.nb); mv(p.bmin); mv(p.bmax); mv(p.wmax); mv(p.U); mv(p.E);
            mv(p.mask); mv(p.flag); mv(p.kept); mv(p.cnt); mv(p.rowflag); mv(p.ids);
            mv(p.st_row); mv(p.st_band); mv(p.st_kmesh); mv(p.st_mlo); mv(p.st_mhi); mv(p.P1);
            mv(p.gamma);
        }
        Arena rar(P->mem + P->mem_bytes, run_bytes);
        P->mem_bytes += run_bytes;
        for (auto& p : P->sp) {
            if (!in_graph(p)) continue;
            p.F = rar.take<cf>((size_t)p.states * p.rp_pad * p.nc_pad);
            p.partial = rar.take<double>((size_t)p.states * p.n_qtiles);
        }
        P->d_desc = rar.take<SysDesc>(n_sys);
        P->d_tasks = rar.take<BTask>(tasks.size());
        P->d_head = rar.take<int>(kBatchedShapes);
        P->G = rar.take<cf>(g_max);
        std::vector<SysDesc> desc(n_sys);
        for (int i = 0; i < n_sys; ++i) fill_desc(P->sp[i], desc[i]);
        HIPCHK(h, hipMemcpy(P->d_desc, desc.data(), sizeof(SysDesc) * n_sys, hipMemcpyHostToDevice));
        if (!tasks.empty())
            HIPCHK(h, hipMemcpy(P->d_tasks, tasks.data(), sizeof(BTask) * tasks.size(),
                                hipMemcpyHostToDevice));
        for (int sh = 0; sh < kBatchedShapes; ++sh) {
            if (!P->n_tasks_shape[sh]) continue;
            P->n_wg_shape[sh] = persistent_wgs(P->lds_shape[sh]);
            // kernel attribute set outside the capture
            HIPCHK(h, prepare_batched_rates(sh, P->lds_shape[sh]));
        }

        // ---- capture: stage 1 + folds, persistent rate kernel, reductions ----
        HIPCHK(h, hipStreamCreate(&P->cs));
        HIPCHK(h, hipStreamBeginCapture(P->cs, hipStreamCaptureModeRelaxed));
        for (auto& p : P->sp) {
            if (!in_graph(p)) continue;
            enqueue_stage1(h, p, P->G, 0, p.states, p.F, p.nc_pad, P->cs);
        }
        HIPCHK(h, launch_zero(P->d_head, sizeof(int) * kBatchedShapes, P->cs));
        for (int sh = 0, t0 = 0; sh < kBatchedShapes; t0 += P->n_tasks_shape[sh++])
            if (P->n_tasks_shape[sh])
                HIPCHK(h, launch_batched_rates(sh, P->d_desc, P->d_tasks + t0, P->n_tasks_shape[sh],
                                               P->d_head + sh, P->n_wg_shape[sh],
                                               P->lds_shape[sh], P->cs));
        for (auto& p : P->sp) {
            if (!in_graph(p)) continue;
            const double scale = 2.0 * kPi / (std::sqrt(kPi) * p.sigma) / (double)p.N;
            HIPCHK(h, launch_zero(p.gamma, (size_t)p.rows * p.nW * sizeof(double), P->cs));
            HIPCHK(h, launch_reduce_partials(p.partial, p.states, p.n_qtiles, p.st_row, p.st_band,
                                             p.nW, scale, p.gamma, P->cs));
        }
        HIPCHK(h, hipStreamEndCapture(P->cs, &P->graph));
        HIPCHK(h, hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
        *plan_out = P;
    });
    if (st != PHOEBE_OK) {
        if (P && P->cs) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(P->cs, &g);
            if (g) (void)hipGraphDestroy(g);
        }
        destroy_plan(P);
    }
    return st;
}

phoebe_status phoebe_gpu_batched_run(void* plan, double* const* gamma_out, void* stream) {
    Plan* P = static_cast<Plan*>(plan);
    if (!P) return PHOEBE_E_INVALID;
    Handle* h = P->h;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        HIPCHK(h, hipSetDevice(h->device));
        HIPCHK(h, hipGraphLaunch(P->exec, s));
        for (int i = 0; i < P->n_sys; ++i) {
            SysPlan& p = P->sp[i];
            if (!p.plain || p.rows == 0) continue;
            // the plain rate call (its factorised mesh sums) straight into the caller's rows,
            // on the band and phonon tables the plan built
            double* dst = gamma_out && gamma_out[i] ? gamma_out[i] : p.gamma;
            const int32_t m[3] = {p.mesh.n0, p.mesh.n1, p.mesh.n2};
            int64_t nk = 0;
            const PresetTables pt{p.eps, p.U, p.omega, p.E, p.nb};
            h->preset = &pt;
            const phoebe_status st2 =
                phoebe_gpu_scatter_rates(h, p.sys, m, m, nullptr, 0, nullptr, nullptr, nullptr,
                                         &p.par, PHOEBE_FP32, dst, nullptr, nullptr, &nk, s);
            h->preset = nullptr;
            if (st2 != PHOEBE_OK) throw Fail{st2};
            REQUIRE(h, nk == p.rows, "system %d: %lld kept k, the plan found %lld", i,
                    (long long)nk, (long long)p.rows);
        }
        if (gamma_out) {
            for (int i = 0; i < P->n_sys; ++i) {
                const SysPlan& p = P->sp[i];
                if (!gamma_out[i] || p.rows == 0 || p.plain) continue;
                HIPCHK(h, hipMemcpyAsync(gamma_out[i], p.gamma, (size_t)p.rows * p.nW * sizeof(double),
                                         hipMemcpyDeviceToDevice, s));
            }
        }
    });
}

phoebe_status phoebe_gpu_batched_info(void* plan, int32_t sys, int32_t* tq, int32_t* tn,
                                      int64_t* n_states, int64_t* n_tasks, double* tune_ms) {
    Plan* P = static_cast<Plan*>(plan);
    if (!P || sys < 0 || sys >= P->n_sys) return PHOEBE_E_INVALID;
    const SysPlan& p = P->sp[sys];
    if (tq) *tq = p.tq;
    if (tn) *tn = p.tn;
    if (n_states) *n_states = p.states;
    if (n_tasks) *n_tasks = P->n_tasks;
    if (tune_ms) *tune_ms = P->tune_ms;
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_batched_destroy(void* plan) {
    Plan* P = static_cast<Plan*>(plan);
    if (!P) return PHOEBE_OK;
    (void)hipSetDevice(P->h->device);
    (void)hipDeviceSynchronize();
    destroy_plan(P);
    return PHOEBE_OK;
}

}  // extern "C"
