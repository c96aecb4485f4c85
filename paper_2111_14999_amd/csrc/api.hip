// C ABI of the library: argument validation, workspace, orchestration of the
// kernels for the band structure, the coupling interpolation and the rates.
#include <array>

#include "ext.hpp"
#include "host.hpp"

using namespace phx;

namespace phx {
std::string g_create_error;
}

extern "C" {

int32_t phoebe_gpu_abi_version(void) { return PHOEBE_GPU_ABI_VERSION; }

phoebe_status phoebe_gpu_create(int device, size_t budget, void** handle) {
    if (!handle) {
        g_create_error = "handle out-pointer is NULL";
        return PHOEBE_E_INVALID;
    }
    *handle = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetDeviceCount failed: ") + hipGetErrorString(e);
        return PHOEBE_E_DEVICE;
    }
    if (device < 0 || device >= count) {
        g_create_error = "device index out of range";
        return PHOEBE_E_INVALID;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipSetDevice failed: ") + hipGetErrorString(e);
        return PHOEBE_E_DEVICE;
    }
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        e = hipMemGetInfo(&fr, &tot);
        if (e != hipSuccess) {
            g_create_error = std::string("hipMemGetInfo failed: ") + hipGetErrorString(e);
            return PHOEBE_E_DEVICE;
        }
        budget = (size_t)(0.9 * (double)fr);
    }
    Handle* h = new (std::nothrow) Handle();
    if (!h) {
        g_create_error = "host allocation failed";
        return PHOEBE_E_NOMEM;
    }
    h->device = device;
    h->budget = budget;
    // the static scratch of phoebe_gpu_scatter_rates_noalloc on this device; a failed
    // lookup leaves it NULL and only that entry point reports it
    if (noalloc_scratch_init(device, &h->scratch) != hipSuccess) h->scratch = nullptr;
    *handle = h;
    g_create_error.clear();
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_destroy(void* handle) {
    if (!handle) return PHOEBE_OK;
    Handle* h = static_cast<Handle*>(handle);
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    for (auto& t : h->pending) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    if (h->ws) (void)hipFree(h->ws);
    if (h->dflag) (void)hipFree(h->dflag);
    if (h->tc.mem) (void)hipFree(h->tc.mem);
    delete h;
    return PHOEBE_OK;
}

const char* phoebe_gpu_last_error(void* handle) {
    if (!handle) return g_create_error.c_str();
    return static_cast<Handle*>(handle)->err.c_str();
}

phoebe_status phoebe_gpu_set_mesh_sum(void* handle, int32_t mode) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    if (mode < PHOEBE_MESH_SUM_AUTO || mode > PHOEBE_MESH_SUM_FACTORED) {
        h->err = "mesh-sum mode out of range";
        return PHOEBE_E_INVALID;
    }
    h->mesh_sum = mode;
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_set_timing(void* handle, int enable) {
    if (!handle) return PHOEBE_E_INVALID;
    static_cast<Handle*>(handle)->timing = enable != 0;
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_reset_timing(void* handle) {
    if (!handle) return PHOEBE_E_INVALID;
    static_cast<Handle*>(handle)->stats.clear();
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_kernel_time(void* handle, const char* name, int64_t* launches,
                                     double* total_ms) {
    if (!handle || !name || !launches || !total_ms) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    *launches = 0;
    *total_ms = 0.0;
    for (auto& k : h->stats)
        if (k.name == name) {
            *launches = k.launches;
            *total_ms = k.total_ms;
        }
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_kernel_bytes(void* handle, const char* name, double* bytes) {
    if (!handle || !name || !bytes) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    *bytes = 0.0;
    for (auto& k : h->stats)
        if (k.name == name) *bytes = k.bytes;
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_electron_bands(void* handle, const phoebe_system* sys,
                                        const double* k_frac, int64_t nk, double* eps_out,
                                        phoebe_c128* u_out, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        check_system(h, sys, true, false, false);
        REQUIRE(h, nk >= 0, "nk < 0");
        if (nk == 0) return;
        REQUIRE(h, k_frac && eps_out, "k_frac/eps_out is NULL");
        REQUIRE(h, sys->n_wannier <= 32, "n_wannier > 32 is not supported");
        HIPCHK(h, hipSetDevice(h->device));
        scan_finite(h, sys, true, false, false, s);
        const int nW = sys->n_wannier;
        auto plan = [&](Arena& ar) {
            int32_t* rh = upload_r(h, ar, sys->rh, sys->n_rh, s);
            cd* U = u_out ? reinterpret_cast<cd*>(u_out) : ar.take<cd>((size_t)nk * nW * nW);
            electron_bands_dev(h, ar, sys, rh, k_frac, nullptr, Mesh{1, 1, 1}, nk, eps_out, U, s);
        };
        Arena dry(nullptr);
        plan(dry);
        ensure_ws(h, dry.used);
        Arena ar(h->ws, h->ws_cap);
        plan(ar);
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipStreamSynchronize(s));  // host lattice lists are read before return
        flush_timing(h, s);
    });
}

phoebe_status phoebe_gpu_phonon_modes(void* handle, const phoebe_system* sys,
                                      const double* q_frac, int64_t nq, double* omega_out,
                                      phoebe_c128* z_out, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        check_system(h, sys, false, true, false);
        REQUIRE(h, nq >= 0, "nq < 0");
        if (nq == 0) return;
        REQUIRE(h, q_frac && omega_out, "q_frac/omega_out is NULL");
        REQUIRE(h, sys->n_atoms <= 10, "more than 10 atoms (30 modes) is not supported");
        HIPCHK(h, hipSetDevice(h->device));
        scan_finite(h, sys, false, true, false, s);
        auto plan = [&](Arena& ar) {
            int32_t* rd = upload_r(h, ar, sys->rd, sys->n_rd, s);
            phonon_dev(h, ar, sys, rd, q_frac, nullptr, Mesh{1, 1, 1}, nq, 0.0, 0.0, omega_out,
                       nullptr, nullptr, reinterpret_cast<cd*>(z_out), s);
        };
        Arena dry(nullptr);
        plan(dry);
        ensure_ws(h, dry.used);
        Arena ar(h->ws, h->ws_cap);
        plan(ar);
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipStreamSynchronize(s));  // host lattice lists are read before return
    });
}

}  // extern "C"

namespace {

// Interpolated g for every (k, q) pair: q_frac (device) a list of nq points, or
// q_frac = NULL and q_mesh (host) the full mesh, nq = N0 N1 N2 points in linear
// order.  On the mesh, FP64 and FP32, where the Rp box is at most half as wide as
// the Rp count, the sum over Rp is taken one axis at a time (the first two by the
// rate path's axis transforms, the last written out row by row): the same sum
// up to the order of the additions, without the dense contraction over Rp.
phoebe_status interp_g_impl(Handle* h, const phoebe_system* sys, const double* k_frac,
                            int64_t nk, const double* q_frac_in, int64_t nq,
                            const int32_t* q_mesh, double omega_min, phoebe_precision prec,
                            phoebe_c128* g_out, double* eps_k, double* eps_kq, double* omega_q,
                            hipStream_t s, const char* name) {
    return run(h, name, [&] {
        check_system(h, sys, true, true, true);
        REQUIRE(h, nk >= 0 && nq >= 0, "negative nk or nq");
        REQUIRE(h, prec >= PHOEBE_FP64 && prec <= PHOEBE_BF16X6, "precision enum out of range");
        REQUIRE(h, std::isfinite(omega_min) && omega_min >= 0.0, "omega_min must be >= 0");
        Mesh qm{1, 1, 1};
        if (q_mesh) {
            REQUIRE(h, q_mesh[0] >= 1 && q_mesh[1] >= 1 && q_mesh[2] >= 1, "q_mesh must be >= 1");
            qm = Mesh{q_mesh[0], q_mesh[1], q_mesh[2]};
            REQUIRE(h, (int64_t)qm.n0 * qm.n1 * qm.n2 <= (int64_t)1 << 26, "q mesh too large");
            nq = (int64_t)qm.n0 * qm.n1 * qm.n2;
        }
        if (nk == 0 || nq == 0) return;
        REQUIRE(h, k_frac && (q_frac_in || q_mesh) && g_out, "k_frac/q_frac/g_out is NULL");
        REQUIRE(h, nk * nq <= 4000000, "nk * nq above 4e6 pairs: split the call");
        const int nW = sys->n_wannier, nm = 3 * sys->n_atoms;
        if (nW > 32 || nm > 32) {
            set_err(h, "nW > 32 or nModes > 32 is not supported");
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        const bool lowp = prec != PHOEBE_FP64;
        const size_t el = lowp ? sizeof(cf) : sizeof(cd);
        const bool polar = sys->polar != nullptr;
        if (polar) check_polar(h, sys);
        HIPCHK(h, hipSetDevice(h->device));
        scan_finite(h, sys, true, true, true, s);
        const int n_re = sys->n_re, n_rp = sys->n_rp;
        const int64_t NC3 = (int64_t)nm * nW * nW;
        const int64_t npair = nk * nq;
        const int64_t kb = std::min<int64_t>(nk, 64);
        // factorised sum over Rp on the mesh (see above)
        const int rmax_p = rmax_of(sys->rp, n_rp);
        const int Wbox = 2 * rmax_p + 1;
        const bool fact = q_mesh && (prec == PHOEBE_FP64 || prec == PHOEBE_FP32) && Wbox <= 31 &&
                          2 * Wbox <= n_rp;
        const int64_t NL = (int64_t)qm.n1 * qm.n2;
        const int64_t ncp = (NC3 + 63) / 64 * 64;  // F and T columns, 64-wide blocks
        const bool axes_fused = fact && axis_transforms_fused(rmax_p, (int)ncp, lowp);
        // FP64 with nW, nModes <= 16: the last axis feeds the rotation in registers
        const bool fused_rot = fact && !lowp && axis0_rotate_supported(rmax_p, nW, nm);
        // q rows per rotation chunk (whole q0 planes on the mesh)
        const int64_t planes = fact ? std::max<int64_t>(1, 65536 / NL) : 0;
        const int64_t qchunk = fact ? std::min<int64_t>(nq, planes * NL) : std::min<int64_t>(nq, 65536);
        std::vector<double> qf_h;
        std::vector<int32_t> box;
        if (q_mesh) {
            qf_h.resize((size_t)nq * 3);
            for (int64_t q = 0; q < nq; ++q) {
                int i0, i1, i2;
                mesh_triple(q, qm, i0, i1, i2);
                qf_h[3 * q] = (double)i0 / qm.n0;
                qf_h[3 * q + 1] = (double)i1 / qm.n1;
                qf_h[3 * q + 2] = (double)i2 / qm.n2;
            }
        }
        // k points on the q mesh: every k + q is a mesh point, so the bands at the pairs
        // are the mesh's (one eigensolve per mesh point, gathered per pair)
        std::vector<int32_t> kidx_h;
        if (q_mesh) {
            std::vector<double> kh((size_t)nk * 3);
            HIPCHK(h, hipMemcpyAsync(kh.data(), k_frac, sizeof(double) * kh.size(),
                                     hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            const int Nd[3] = {qm.n0, qm.n1, qm.n2};
            kidx_h.resize(nk);
            for (int64_t i = 0; i < nk && !kidx_h.empty(); ++i) {
                int id[3];
                for (int d = 0; d < 3; ++d) {
                    const double x = kh[3 * i + d] * Nd[d];
                    const double r = std::nearbyint(x);
                    if (!(std::fabs(x - r) <= 1e-9 * std::max(1.0, std::fabs(x)))) {
                        kidx_h.clear();
                        break;
                    }
                    id[d] = (int)(((int64_t)r % Nd[d] + Nd[d]) % Nd[d]);
                }
                if (!kidx_h.empty()) kidx_h[i] = (int32_t)mesh_linear(id[0], id[1], id[2], qm);
            }
        }
        const bool k_on_mesh = !kidx_h.empty();
        if (fact) {
            box.assign((size_t)Wbox * Wbox * Wbox, -1);
            for (int i = 0; i < n_rp; ++i) {
                const int64_t b = ((int64_t)(sys->rp[3 * i] + rmax_p) * Wbox +
                                   (sys->rp[3 * i + 1] + rmax_p)) * Wbox +
                                  (sys->rp[3 * i + 2] + rmax_p);
                REQUIRE(h, box[b] < 0, "Rp list holds a vector twice");
                box[b] = i;
            }
        }
        auto plan = [&](Arena& ar) {
            int32_t* rh = upload_r(h, ar, sys->rh, sys->n_rh, s);
            int32_t* rd = upload_r(h, ar, sys->rd, sys->n_rd, s);
            int32_t* re = upload_r(h, ar, sys->re, n_re, s);
            int32_t* rp = upload_r(h, ar, sys->rp, n_rp, s);
            double* qfd = q_mesh ? ar.take<double>((size_t)nq * 3) : nullptr;
            const double* q_frac = q_mesh ? qfd : q_frac_in;
            double* ek = eps_k ? eps_k : ar.take<double>((size_t)nk * nW);
            cd* Uk = ar.take<cd>((size_t)nk * nW * nW);
            double* ekq = eps_kq ? eps_kq : ar.take<double>((size_t)npair * nW);
            cd* Ukq = ar.take<cd>((size_t)npair * nW * nW);
            double* kqf = k_on_mesh ? nullptr : ar.take<double>((size_t)npair * 3);
            double* eps_m = k_on_mesh ? ar.take<double>((size_t)nq * nW) : nullptr;
            cd* U_m = k_on_mesh ? ar.take<cd>((size_t)nq * nW * nW) : nullptr;
            int32_t* kidx_d = k_on_mesh ? ar.take<int32_t>((size_t)nk) : nullptr;
            double* om = omega_q ? omega_q : ar.take<double>((size_t)nq * nm);
            cd* E = ar.take<cd>((size_t)nq * nm * nm);
            cd* Pe = ar.take<cd>((size_t)kb * n_re);
            char* G1 = ar.take<char>((size_t)kb * n_rp * NC3 * el);
            cd* Pp = fact ? nullptr : ar.take<cd>((size_t)nq * n_rp);
            char* F = ar.take<char>((size_t)n_rp * (fact ? ncp : NC3) * el);
            char* X = fused_rot ? nullptr : ar.take<char>((size_t)qchunk * NC3 * el);
            cd* Lq = polar ? ar.take<cd>((size_t)nq * nm) : nullptr;
            double* born = polar ? ar.take<double>((size_t)9 * sys->n_atoms) : nullptr;
            int32_t* box_d = fact ? ar.take<int32_t>(box.size()) : nullptr;
            cd* Pax = fact ? ar.take<cd>((size_t)(qm.n0 + qm.n1 + qm.n2) * Wbox) : nullptr;
            uint32_t* all_lines = fact ? ar.take<uint32_t>((size_t)NL) : nullptr;
            char* T1 = fact && !axes_fused ? ar.take<char>((size_t)Wbox * Wbox * qm.n2 * ncp * el)
                                           : nullptr;
            char* T2 = fact ? ar.take<char>((size_t)Wbox * NL * ncp * el) : nullptr;
            if (ar.base && q_mesh)
                HIPCHK(h, hipMemcpyAsync(qfd, qf_h.data(), sizeof(double) * qf_h.size(),
                                         hipMemcpyHostToDevice, s));
            {
                Arena sub = ar;  // band scratch, reused after the tables are built
                electron_bands_dev(h, sub, sys, rh, k_frac, nullptr, Mesh{1, 1, 1}, nk, ek, Uk, s);
                Arena sub2 = ar;
                if (k_on_mesh) {
                    electron_bands_dev(h, sub2, sys, rh, nullptr, nullptr, qm, nq, eps_m, U_m, s);
                    if (ar.base) {
                        HIPCHK(h, hipMemcpyAsync(kidx_d, kidx_h.data(), sizeof(int32_t) * nk,
                                                 hipMemcpyHostToDevice, s));
                        HIPCHK(h, launch_gather_kq_bands(eps_m, U_m, nW, qm, kidx_d, nk, nq, ekq,
                                                         Ukq, s));
                    }
                } else {
                    if (ar.base) HIPCHK(h, launch_kq_points(k_frac, nk, q_frac, nq, kqf, s));
                    electron_bands_dev(h, sub2, sys, rh, kqf, nullptr, Mesh{1, 1, 1}, npair, ekq,
                                       Ukq, s);
                }
                Arena sub3 = ar;
                phonon_dev(h, sub3, sys, rd, q_frac, nullptr, Mesh{1, 1, 1}, nq, omega_min, 0.0,
                           om, E, nullptr, nullptr, s);
                ar.used = std::max(std::max(sub.used, sub2.used), sub3.used);
            }
            if (!ar.base) return;
            if (polar) {
                HIPCHK(h, hipMemcpyAsync(born, sys->polar->born, sizeof(double) * 9 * sys->n_atoms,
                                         hipMemcpyHostToDevice, s));
                HIPCHK(h, launch_polar_factor(q_frac, Mesh{1, 1, 1}, nq, E, nm, polar_dev(sys, born),
                                              Lq, s));
            }
            if (fact) {
                HIPCHK(h, hipMemcpyAsync(box_d, box.data(), sizeof(int32_t) * box.size(),
                                         hipMemcpyHostToDevice, s));
                HIPCHK(h, launch_axis_phases(qm, rmax_p, Pax, s));
                HIPCHK(h, hipMemsetAsync(all_lines, 0xFF, sizeof(uint32_t) * NL, s));  // every line
                // the columns beyond nModes nW^2 stay zero (the fold writes the others)
                if (ncp > NC3) HIPCHK(h, launch_zero(F, (size_t)n_rp * ncp * el, s));
            } else {
                HIPCHK(h, launch_phase_table(q_frac, nullptr, Mesh{1, 1, 1}, nq, rp, n_rp, Pp, n_rp, s));
            }
            for (int64_t k0 = 0; k0 < nk; k0 += kb) {
                const int64_t nb = std::min(kb, nk - k0);
                HIPCHK(h, launch_phase_table(k_frac + 3 * k0, nullptr, Mesh{1, 1, 1}, nb, re, n_re,
                                             Pe, n_re, s));
                Timer t1(h, s, "stage1_phase");
                if (lowp)
                    HIPCHK(h, launch_cgemm_lp(prec, Pe, n_re, reinterpret_cast<const cd*>(sys->g_rr),
                                              (int64_t)n_rp * NC3, reinterpret_cast<cf*>(G1),
                                              (int64_t)n_rp * NC3, nb, (int64_t)n_rp * NC3, n_re, s));
                else
                    HIPCHK(h, launch_zgemm(Pe, n_re, reinterpret_cast<const cd*>(sys->g_rr),
                                           (int64_t)n_rp * NC3, reinterpret_cast<cd*>(G1),
                                           (int64_t)n_rp * NC3, nb, (int64_t)n_rp * NC3, n_re, s));
                t1.done();
                for (int64_t i = 0; i < nb; ++i) {
                    const int64_t k = k0 + i;
                    const int64_t ldf = fact ? ncp : NC3;
                    if (lowp)
                        HIPCHK(h, launch_fold_all_lp(reinterpret_cast<const cf*>(G1) + i * n_rp * NC3,
                                                     Uk + k * nW * nW, n_rp, nm, nW,
                                                     reinterpret_cast<cf*>(F), s, ldf));
                    else
                        HIPCHK(h, launch_fold_all(reinterpret_cast<const cd*>(G1) + i * n_rp * NC3,
                                                  Uk + k * nW * nW, n_rp, nm, nW,
                                                  reinterpret_cast<cd*>(F), s, ldf));
                    if (fact) {  // first two Rp axes for every line of the mesh
                        Timer ta(h, s, "interp_axes");
                        if (lowp)
                            HIPCHK(h, launch_axis_transforms_f32(
                                          reinterpret_cast<const cf*>(F), n_rp, (int)ncp, box_d,
                                          rmax_p, qm, Pax, 1, all_lines, reinterpret_cast<cf*>(T1),
                                          reinterpret_cast<cf*>(T2), s));
                        else
                            HIPCHK(h, launch_axis_transforms(
                                          reinterpret_cast<const cd*>(F), n_rp, (int)ncp, box_d,
                                          rmax_p, qm, Pax, 1, all_lines, reinterpret_cast<cd*>(T1),
                                          reinterpret_cast<cd*>(T2), s));
                        ta.done();
                    }
                    if (fused_rot) {  // last axis and rotation together, every q of this k
                        cd* gk = reinterpret_cast<cd*>(g_out) + k * nq * NC3;
                        Timer tx(h, s, "interp_axis0_rotate");
                        HIPCHK(h, launch_axis0_rotate(reinterpret_cast<const cd*>(T2), qm, (int)ncp,
                                                      rmax_p, Pax, E, Ukq + k * nq * nW * nW, nW,
                                                      nm, gk, s));
                        tx.done();
                        if (polar)
                            HIPCHK(h, launch_polar_add_g(gk, nq, Uk + k * nW * nW,
                                                         Ukq + k * nq * nW * nW, Lq, nW, nm, s));
                        continue;
                    }
                    for (int64_t q0 = 0; q0 < nq; q0 += qchunk) {
                        const int64_t nqc = std::min(qchunk, nq - q0);
                        cd* gk = reinterpret_cast<cd*>(g_out) + (k * nq + q0) * NC3;
                        if (fact) {  // last axis: X rows of the chunk's q0 planes
                            Timer tx(h, s, "interp_axis0");
                            const int pa = (int)(q0 / NL), pb = (int)((q0 + nqc) / NL);
                            if (lowp)
                                HIPCHK(h, launch_axis0_out_f32(reinterpret_cast<const cf*>(T2), qm,
                                                               (int)ncp, (int)NC3, rmax_p, Pax, pa,
                                                               pb, reinterpret_cast<cf*>(X), NC3, s));
                            else
                                HIPCHK(h, launch_axis0_out(reinterpret_cast<const cd*>(T2), qm,
                                                           (int)ncp, (int)NC3, rmax_p, Pax, pa, pb,
                                                           reinterpret_cast<cd*>(X), NC3, s));
                            tx.done();
                        } else if (lowp) {
                            HIPCHK(h, launch_cgemm_lp_cf(prec, Pp + q0 * n_rp, n_rp,
                                                         reinterpret_cast<const cf*>(F), NC3,
                                                         reinterpret_cast<cf*>(X), NC3, nqc, NC3,
                                                         n_rp, s));
                        } else {
                            HIPCHK(h, launch_zgemm(Pp + q0 * n_rp, n_rp, reinterpret_cast<const cd*>(F),
                                                   NC3, reinterpret_cast<cd*>(X), NC3, nqc, NC3, n_rp,
                                                   s));
                        }
                        if (lowp)
                            HIPCHK(h, launch_rotate_g_lp(reinterpret_cast<const cf*>(X), nqc,
                                                         Ukq + (k * nq + q0) * nW * nW,
                                                         E + q0 * nm * nm, nW, nm, gk, s));
                        else
                            HIPCHK(h, launch_rotate_g(reinterpret_cast<const cd*>(X), nqc,
                                                      Uk + k * nW * nW, Ukq + (k * nq + q0) * nW * nW,
                                                      E + q0 * nm * nm, nW, nm, gk, s));
                        if (polar)  // + i L(q, nu) [U_k^dagger U_{k+q}]_{n m}
                            HIPCHK(h, launch_polar_add_g(gk, nqc, Uk + k * nW * nW,
                                                         Ukq + (k * nq + q0) * nW * nW,
                                                         Lq + q0 * nm, nW, nm, s));
                    }
                }
            }
        };
        Arena dry(nullptr);
        plan(dry);
        ensure_ws(h, dry.used);
        Arena ar(h->ws, h->ws_cap);
        plan(ar);
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipStreamSynchronize(s));  // host lattice lists are read before return
        flush_timing(h, s);
    });
}

}  // namespace

extern "C" {

phoebe_status phoebe_gpu_interp_g(void* handle, const phoebe_system* sys, const double* k_frac,
                                  int64_t nk, const double* q_frac, int64_t nq, double omega_min,
                                  phoebe_precision prec, phoebe_c128* g_out, double* eps_k,
                                  double* eps_kq, double* omega_q, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    return interp_g_impl(static_cast<Handle*>(handle), sys, k_frac, nk, q_frac, nq, nullptr,
                         omega_min, prec, g_out, eps_k, eps_kq, omega_q,
                         static_cast<hipStream_t>(stream), __func__);
}

phoebe_status phoebe_gpu_interp_g_mesh(void* handle, const phoebe_system* sys,
                                       const double* k_frac, int64_t nk, const int32_t q_mesh[3],
                                       double omega_min, phoebe_precision prec, phoebe_c128* g_out,
                                       double* eps_k, double* eps_kq, double* omega_q,
                                       void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    if (!q_mesh) {
        h->err = "q_mesh is NULL";
        return PHOEBE_E_INVALID;
    }
    return interp_g_impl(h, sys, k_frac, nk, nullptr, 0, q_mesh, omega_min, prec, g_out, eps_k,
                         eps_kq, omega_q, static_cast<hipStream_t>(stream), __func__);
}

}  // extern "C"

// Rate path; with `terms` (FP64, full q mesh only) it also writes each kept
// state's per-(q, mode) terms and the state list.
static phoebe_status scatter_rates_impl(void* handle, const phoebe_system* sys,
                                        const int32_t mesh_in[3], const int32_t* q_mesh_in,
                                        double* lw_out, const int32_t* k_idx, int64_t nk,
                                        const int64_t* q_off, const int32_t* q_idx,
                                        const double* q_w, const phoebe_rate_params* par,
                                        phoebe_precision prec, double* gamma_out,
                                        uint8_t* band_mask, int32_t* kept_k_out,
                                        int64_t* n_kept_out, double* terms, int32_t* st_row_out,
                                        int32_t* st_band_out, int64_t* n_states_out,
                                        double* dweights, bool rates, int64_t state_cap,
                                        void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        check_system(h, sys, true, true, true);
        REQUIRE(h, mesh_in != nullptr, "mesh is NULL");
        REQUIRE(h, mesh_in[0] >= 1 && mesh_in[1] >= 1 && mesh_in[2] >= 1, "mesh must be >= 1");
        REQUIRE(h, par != nullptr, "rate parameters are NULL");
        REQUIRE(h, std::isfinite(par->sigma) && par->sigma > 0.0, "sigma must be > 0");
        REQUIRE(h, std::isfinite(par->kT) && par->kT > 0.0, "kT must be > 0");
        REQUIRE(h, std::isfinite(par->mu), "mu must be finite");
        REQUIRE(h, !std::isnan(par->win_lo) && !std::isnan(par->win_hi), "window is NaN");
        REQUIRE(h, std::isfinite(par->omega_min) && par->omega_min >= 0.0, "omega_min must be >= 0");
        REQUIRE(h, prec >= PHOEBE_FP64 && prec <= PHOEBE_BF16X6, "precision enum out of range");
        REQUIRE(h, gamma_out != nullptr, "gamma_out is NULL");
        REQUIRE(h, k_idx != nullptr || nk == 0, "nk must be 0 when k_idx is NULL");
        REQUIRE(h, nk >= 0, "nk < 0");
        REQUIRE(h, (q_off == nullptr) == (q_idx == nullptr) && (q_off == nullptr) == (q_w == nullptr),
                "q_off, q_idx and q_w must be all NULL or all set");
        REQUIRE(h, q_off == nullptr || k_idx != nullptr, "explicit q lists need explicit k_idx");
        REQUIRE(h, terms == nullptr || (prec == PHOEBE_FP64 && q_off == nullptr && k_idx != nullptr),
                "per-term output needs FP64, explicit k_idx and the full q mesh");
        REQUIRE(h, dweights == nullptr || (q_off == nullptr && k_idx != nullptr),
                "smearing weights need explicit k_idx and the full q mesh");
        REQUIRE(h, par->smearing == PHOEBE_SMEAR_GAUSSIAN || par->smearing == PHOEBE_SMEAR_ADAPTIVE,
                "smearing enum out of range");
        const bool adaptive = par->smearing == PHOEBE_SMEAR_ADAPTIVE;
        REQUIRE(h, !adaptive || (std::isfinite(par->adaptive_scale) && par->adaptive_scale > 0.0),
                "adaptive_scale must be > 0");
        const bool polar = sys->polar != nullptr;
        if (polar) check_polar(h, sys);
        REQUIRE(h, lw_out == nullptr || (k_idx == nullptr && q_off == nullptr),
                "the linewidth sums over every kept k of the full meshes");
        if (q_mesh_in) {
            REQUIRE(h, q_mesh_in[0] >= 1 && q_mesh_in[1] >= 1 && q_mesh_in[2] >= 1,
                    "q mesh must be >= 1");
            if (q_mesh_in[0] != mesh_in[0] || q_mesh_in[1] != mesh_in[1] ||
                q_mesh_in[2] != mesh_in[2]) {
                set_err(h, "a q mesh different from the k mesh is not supported (k + q must be a "
                           "point of the k mesh)");
                throw Fail{PHOEBE_E_UNSUPPORTED};
            }
        }
        const bool ext = adaptive || polar || lw_out != nullptr;
        if (ext && prec != PHOEBE_FP64) {
            set_err(h, "polar coupling, adaptive smearing and the linewidth need FP64");
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        if (adaptive && (terms || dweights)) {
            set_err(h, "per-term outputs and smearing weights take the fixed Gaussian width");
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        const Mesh mesh{mesh_in[0], mesh_in[1], mesh_in[2]};
        const int64_t N = (int64_t)mesh.n0 * mesh.n1 * mesh.n2;
        REQUIRE(h, N <= (int64_t)1 << 30, "mesh too large");
        const int nW = sys->n_wannier, nm = 3 * sys->n_atoms;
        if (nW > 32 || nm > 32) {
            set_err(h, "nW > 32 or nModes > 32 is not supported");
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        const bool lowp = prec != PHOEBE_FP64;
        int tq = 0, tn = 0;
        const int nc_direct = lowp ? stage2_lp_config(nm, nW, &tq, &tn) : stage2_config(nm, nW, &tq, &tn);
        if (nc_direct < 0) {
            set_err(h, "no stage-2 tiling for nModes*nW = %d", nm * nW);
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        const int rmax_p = rmax_of(sys->rp, sys->n_rp);
        REQUIRE(h, rmax_p <= 100, "|Rp| components above 100 are not supported");
        // Full-mesh FP64 sums may take the per-axis factorised form (see
        // launch_axis_transforms / launch_line_rates).
        const int Wbox = 2 * rmax_p + 1;
        const int nc_line = line_rates_ncpad(nm, nW);
        const int64_t NL = (int64_t)mesh.n1 * mesh.n2;
        const bool can_factor = (prec == PHOEBE_FP64 || prec == PHOEBE_FP32) && q_off == nullptr &&
                                Wbox <= 31 && nc_line > 0 && NL <= 65535 && mesh.n0 <= 1024 &&
                                line_rates_lds(Wbox, mesh.n0, nm, lowp, lw_out != nullptr) <=
                                    64 * 1024;
        if (h->mesh_sum == PHOEBE_MESH_SUM_FACTORED && !can_factor) {
            set_err(h, "the factorised mesh sum needs FP64 or FP32, the full q mesh, |Rp| <= 15, "
                       "nW <= 32, nModes <= 32, N0 <= 1024 and N1*N2 <= 65535");
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        HIPCHK(h, hipSetDevice(h->device));
        scan_finite(h, sys, true, true, true, s);
        const bool factored = can_factor && (h->mesh_sum == PHOEBE_MESH_SUM_FACTORED ||
                                             (h->mesh_sum == PHOEBE_MESH_SUM_AUTO &&
                                              2 * Wbox <= sys->n_rp));
        // stage-2 operand columns: sa*nW + b (direct), sa*16 + b (factorised, nW <= 16) or
        // sa*32 + b (factorised, nW <= 32)
        const int nc_pad = factored ? nc_line : nc_direct;
        const int cw = factored ? (nW <= 16 ? 16 : 32) : nW;
        HIPCHK(h, hipSetDevice(h->device));
        const int n_re = sys->n_re, n_rp = sys->n_rp;
        // K padding of the stage-2 operand: 4 (K of the f64/f32 MFMA) or 32 (bf16)
        const bool bf16 = prec == PHOEBE_BF16X3 || prec == PHOEBE_BF16X6;
        if (bf16 && tn > 8) {
            set_err(h, "split-BF16 contractions take nModes*nW <= 512 (here %d)", nm * nW);
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        const int rp_pad = bf16 ? (n_rp + 31) & ~31 : (n_rp + 3) & ~3;
        const int64_t NC2 = (int64_t)n_rp * nm * nW * nW;
        // bytes of one stage-1 element and of one stage-2 operand element
        const size_t g_elem = lowp ? sizeof(cf) : sizeof(cd);
        const size_t f_elem = prec == PHOEBE_FP64 ? sizeof(cd)
                              : prec == PHOEBE_FP32 ? sizeof(cf)
                              : prec == PHOEBE_BF16X3 ? 4 * sizeof(uint16_t) : 6 * sizeof(uint16_t);
        if (lowp && stage2_lp_lds(prec, tq, rmax_p, rp_pad, nc_pad, nm, nW, false) > 159 * 1024) {
            set_err(h, "stage-2 tile does not fit in LDS");
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        // kept k points per stage-1 batch: G and F of a batch stay under 8 GB each
        // Stage 1 takes the same per-axis factorisation over the Re box when the
        // mesh sum is factorised (launch_re_axes); its batches are larger, limited
        // by the distinct k0 and (k0, k1) values they hold (see below).
        const int rmax_e = rmax_of(sys->re, n_re);
        const int We = 2 * rmax_e + 1;
        const bool re_fact = factored && rmax_e <= 15 &&
                             re_axes_lds(rmax_e, lowp) <= 160 * 1024 &&
                             (h->mesh_sum == PHOEBE_MESH_SUM_FACTORED || 2 * We <= n_re);
        constexpr int kD0Max = 8, kD01Max = 256;
        // nW = 16: the pair and k steps of stage 1 apply the U_k fold themselves and
        // write F; G (nW times larger) never reaches HBM
        const bool fold_fused = re_fact && nW == 16 && cw == 16;
        int BK = re_fact ? 256 : 64;
        while (BK > 16 && ((double)BK * NC2 * g_elem > 8e9 ||
                           (double)BK * nW * rp_pad * nc_pad * f_elem > 8e9))
            BK /= 2;
        const int BQ = 16 * tq;
        // states per factorised sub-batch: T1 + T2 of a sub-batch stay under 16 GB or a
        // quarter of the workspace budget, whichever is less (T2 alone where both Rp
        // axes run in one pass and T1 is not used); larger sub-batches mean fewer,
        // longer launches of the axis and line kernels
        const bool axes_fused = factored && axis_transforms_fused(rmax_p, nc_pad, lowp);
        const size_t t12_state =
            ((axes_fused ? 0 : (size_t)Wbox * Wbox * mesh.n2) + (size_t)Wbox * NL) * nc_pad * g_elem;
        const int n0_line = mesh.n0;
        const double sub_cap = std::min(16e9, 0.25 * (double)h->budget);
        const int nsb = factored ? (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)BK * nW,
                                                      (int64_t)(sub_cap / (double)t12_state)))
                                 : 0;

        // q-list lengths (host) for the tile count
        int64_t max_list = N;
        std::vector<int64_t> qoff_h;
        if (q_off) {
            qoff_h.resize(nk + 1);
            HIPCHK(h, hipMemcpyAsync(qoff_h.data(), q_off, sizeof(int64_t) * (nk + 1),
                                     hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            max_list = 0;
            REQUIRE(h, qoff_h[0] >= 0, "q_off[0] < 0");
            for (int64_t i = 0; i < nk; ++i) {
                REQUIRE(h, qoff_h[i + 1] >= qoff_h[i], "q_off is not non-decreasing");
                max_list = std::max(max_list, qoff_h[i + 1] - qoff_h[i]);
            }
            const int64_t total = qoff_h[nk];
            if (total > 0) {
                std::vector<int32_t> qh(total);
                HIPCHK(h, hipMemcpyAsync(qh.data(), q_idx, sizeof(int32_t) * total,
                                         hipMemcpyDeviceToHost, s));
                HIPCHK(h, hipStreamSynchronize(s));
                for (int64_t i = 0; i < total; ++i)
                    REQUIRE(h, qh[i] >= 0 && qh[i] < N, "q_idx[%lld] = %d is not a mesh index",
                            (long long)i, qh[i]);
            }
        }
        const int n_qtiles = factored ? (int)NL : (int)std::max<int64_t>(1, (max_list + BQ - 1) / BQ);

        // ---- phase A: tables, window, states (sized for the whole mesh) ----
        struct Tables {
            int32_t *rh, *rd, *re, *rp, *rp_packed;
            double *eps, *focc, *omega, *nb, *bmin, *bmax, *wmax;
            cd *U, *E;
            uint8_t* mask;
            int32_t *flag, *kept, *cnt, *rowflag, *ids;
            int32_t *st_row, *st_band, *st_kmesh, *st_mlo, *st_mhi;
            int32_t *box_rp, *box_re;
            cd *Pax, *Pre;
            cd* Lpol;            // polar factor [N, nm]
            double* born;        // Born charges [nat, 3, 3]
            double *vel, *vmax;  // group velocities [N, nW, 3], per-axis max |v| [3]
            int32_t* vbad;
            double* lwacc;       // linewidth sums [N, nm]
        } T{};
        const int64_t rows_cap = k_idx ? nk : N;
        auto plan_tables = [&](Arena& ar) {
            T.rh = upload_r(h, ar, sys->rh, sys->n_rh, s);
            T.rd = upload_r(h, ar, sys->rd, sys->n_rd, s);
            T.re = upload_r(h, ar, sys->re, n_re, s);
            T.rp = upload_r(h, ar, sys->rp, n_rp, s);
            T.rp_packed = ar.take<int32_t>(n_rp);
            T.eps = ar.take<double>((size_t)N * nW);
            T.focc = ar.take<double>((size_t)N * nW);
            T.U = ar.take<cd>((size_t)N * nW * nW);
            T.omega = ar.take<double>((size_t)N * nm);
            T.nb = ar.take<double>((size_t)N * nm);
            T.E = ar.take<cd>((size_t)N * nm * nm);
            T.bmin = ar.take<double>(nW);
            T.bmax = ar.take<double>(nW);
            T.wmax = ar.take<double>(1);
            T.mask = ar.take<uint8_t>((size_t)N * nW);
            T.flag = ar.take<int32_t>(N);
            T.kept = ar.take<int32_t>(N);
            T.cnt = ar.take<int32_t>(2);
            T.rowflag = ar.take<int32_t>((size_t)rows_cap * nW);
            T.ids = ar.take<int32_t>((size_t)rows_cap * nW);
            T.st_row = ar.take<int32_t>((size_t)rows_cap * nW);
            T.st_band = ar.take<int32_t>((size_t)rows_cap * nW);
            T.st_kmesh = ar.take<int32_t>((size_t)rows_cap * nW);
            T.st_mlo = ar.take<int32_t>((size_t)rows_cap * nW);
            T.st_mhi = ar.take<int32_t>((size_t)rows_cap * nW);
            if (factored) {
                T.box_rp = ar.take<int32_t>((size_t)Wbox * Wbox * Wbox);
                T.Pax = ar.take<cd>((size_t)(mesh.n0 + mesh.n1 + mesh.n2) * Wbox);
            }
            if (re_fact) {
                T.box_re = ar.take<int32_t>((size_t)We * We * We);
                T.Pre = ar.take<cd>((size_t)(mesh.n0 + mesh.n1 + mesh.n2) * We);
            }
            if (polar) {
                T.Lpol = ar.take<cd>((size_t)N * nm);
                T.born = ar.take<double>((size_t)9 * sys->n_atoms);
            }
            if (adaptive) {
                T.vel = ar.take<double>((size_t)N * nW * 3);
                T.vmax = ar.take<double>(4);
                T.vbad = ar.take<int32_t>(1);
            }
            if (lw_out) T.lwacc = ar.take<double>((size_t)N * nm);
        };
        // band scratch is carved after the tables and reused by the batches
        size_t tables_end = 0, scratch_bands = 0;
        {
            Arena dry(nullptr);
            plan_tables(dry);
            tables_end = dry.used;
            Arena d1 = dry, d2 = dry;
            electron_bands_dev(h, d1, sys, nullptr, nullptr, nullptr, mesh, N, nullptr, nullptr, s);
            phonon_dev(h, d2, sys, nullptr, nullptr, nullptr, mesh, N, 0, 0, nullptr, nullptr,
                       nullptr, nullptr, s);
            Arena d3 = dry;
            if (adaptive) velocity_dev(h, d3, sys, nullptr, nullptr, mesh, N, nullptr, nullptr, true,
                                       nullptr, nullptr, s);
            scratch_bands = std::max(std::max(d1.used, d2.used), d3.used) - tables_end;
        }
        // batch buffers (upper bound on the states of a batch: BK * nW)
        const int max_states = BK * nW;
        // Factorised stage 1 keeps the first intermediate T0 either for the k0
        // planes of one batch (g(Re,Rp) is read once per batch) or, when the
        // workspace budget allows it, for every k0 plane of the call (g is read
        // once per call and the batches are no longer limited by their k0 count).
        const size_t plane_bytes = (size_t)We * We * NC2 * g_elem;
        const int64_t planes_cap = std::min<int64_t>(mesh.n0, rows_cap);
        const size_t batch_bytes = 4 * 256 + (size_t)BK * n_re * sizeof(cd) +
                                   (fold_fused ? 0 : (size_t)BK * NC2 * g_elem) +
                                   (size_t)max_states * rp_pad * nc_pad * f_elem +
                                   (size_t)max_states * n_qtiles * sizeof(double) +
                                   (factored ? (size_t)nsb * t12_state + 512 : 0) +
                                   (factored ? (size_t)nsb * NL * (n0_line + 1) * sizeof(uint32_t) +
                                                   // nlive: 2 per sub-batch; sub-batches <= states + batches
                                                   2 * (size_t)(rows_cap * nW + rows_cap + 1) *
                                                       sizeof(uint32_t) + 512
                                             : 0) +
                                   (re_fact ? (size_t)rows_cap * 176 * sizeof(int32_t) + 1024
                                            : 0) +
                                   (lw_out ? (factored ? (size_t)nsb * NL * n0_line
                                                       : (size_t)max_states * N) *
                                                     nm * sizeof(double) + 256
                                           : 0);
        const bool all_planes =
            re_fact && tables_end + std::max(scratch_bands, batch_bytes + planes_cap * plane_bytes) +
                               256 <= h->budget;
        const size_t t0_bytes = re_fact ? (all_planes ? planes_cap : kD0Max) * plane_bytes : 0;
        ensure_ws(h, tables_end + std::max(scratch_bands, batch_bytes + t0_bytes) + 256);
        Arena ar(h->ws, h->ws_cap);
        plan_tables(ar);
        {
            std::vector<int32_t> packed(n_rp);
            for (int i = 0; i < n_rp; ++i)
                packed[i] = (sys->rp[3 * i] + rmax_p) | ((sys->rp[3 * i + 1] + rmax_p) << 8) |
                            ((sys->rp[3 * i + 2] + rmax_p) << 16);
            HIPCHK(h, hipMemcpyAsync(T.rp_packed, packed.data(), sizeof(int32_t) * n_rp,
                                     hipMemcpyHostToDevice, s));
            std::vector<int32_t> box;
            if (factored) {
                // box position ((R0+r) W + R1+r) W + R2+r -> row of F (-1: no such Rp)
                box.assign((size_t)Wbox * Wbox * Wbox, -1);
                for (int i = 0; i < n_rp; ++i) {
                    const int64_t b = ((int64_t)(sys->rp[3 * i] + rmax_p) * Wbox +
                                       (sys->rp[3 * i + 1] + rmax_p)) * Wbox +
                                      (sys->rp[3 * i + 2] + rmax_p);
                    REQUIRE(h, box[b] < 0, "Rp list holds a vector twice");
                    box[b] = i;
                }
                HIPCHK(h, hipMemcpyAsync(T.box_rp, box.data(), sizeof(int32_t) * box.size(),
                                         hipMemcpyHostToDevice, s));
                HIPCHK(h, launch_axis_phases(mesh, rmax_p, T.Pax, s));
            }
            std::vector<int32_t> box_e;
            if (re_fact) {
                // box position of Re -> row of g(Re, Rp) (-1: no such Re)
                box_e.assign((size_t)We * We * We, -1);
                for (int i = 0; i < n_re; ++i) {
                    const int64_t b = ((int64_t)(sys->re[3 * i] + rmax_e) * We +
                                       (sys->re[3 * i + 1] + rmax_e)) * We +
                                      (sys->re[3 * i + 2] + rmax_e);
                    REQUIRE(h, box_e[b] < 0, "Re list holds a vector twice");
                    box_e[b] = i;
                }
                HIPCHK(h, hipMemcpyAsync(T.box_re, box_e.data(), sizeof(int32_t) * box_e.size(),
                                         hipMemcpyHostToDevice, s));
                HIPCHK(h, launch_axis_phases(mesh, rmax_e, T.Pre, s));
            }
            // the host vector must outlive the copy
            HIPCHK(h, hipStreamSynchronize(s));
        }
        if (h->preset) {
            // tables lent by a batched plan for this call (built there with the same routines)
            T.eps = h->preset->eps;
            T.U = h->preset->U;
            T.omega = h->preset->omega;
            T.E = h->preset->E;
            T.nb = h->preset->nb;
        } else {
            // band and phonon tables: from the table cache when it holds this system's
            // tables on this mesh (same inputs, omega_min and kT), else built here
            const size_t b_eps = sizeof(double) * N * nW, b_U = sizeof(cd) * N * nW * nW,
                         b_om = sizeof(double) * N * nm, b_E = sizeof(cd) * N * nm * nm;
            const size_t tc_bytes = b_eps + b_U + 2 * b_om + b_E;
            TableCache& tc = h->tc;
            const bool use_cache = h->table_cache && !h->fixed_ws;
            const std::vector<int32_t> rh_v(sys->rh, sys->rh + 3 * sys->n_rh),
                rd_v(sys->rd, sys->rd + 3 * sys->n_rd);
            const bool hit = use_cache && tc.valid && tc.h_r == sys->h_r &&
                             tc.phi_r == sys->phi_r && tc.mass == sys->mass && tc.nW == nW &&
                             tc.nat == sys->n_atoms && tc.n0 == mesh.n0 && tc.n1 == mesh.n1 &&
                             tc.n2 == mesh.n2 && tc.omega_min == par->omega_min &&
                             tc.kT == par->kT && tc.rh == rh_v && tc.rd == rd_v;
            char* const parts[5] = {(char*)T.eps, (char*)T.U, (char*)T.omega, (char*)T.E,
                                    (char*)T.nb};
            const size_t sizes[5] = {b_eps, b_U, b_om, b_E, b_om};
            if (hit) {
                size_t o = 0;
                for (int i = 0; i < 5; ++i) {
                    HIPCHK(h, hipMemcpyAsync(parts[i], tc.mem + o, sizes[i],
                                             hipMemcpyDeviceToDevice, s));
                    o += sizes[i];
                }
            } else {
                Arena b1 = ar, b2 = ar;
                electron_bands_dev(h, b1, sys, T.rh, nullptr, nullptr, mesh, N, T.eps, T.U, s);
                // the rate kernels read each eigenvector contiguously
                HIPCHK(h, launch_transpose_batch(T.U, N, nW, s));
                phonon_dev(h, b2, sys, T.rd, nullptr, nullptr, mesh, N, par->omega_min, par->kT,
                           T.omega, T.E, T.nb, nullptr, s);
                if (use_cache) {
                    tc.valid = false;
                    if (tc.bytes < tc_bytes) {
                        if (tc.mem) {
                            HIPCHK(h, hipStreamSynchronize(s));
                            char* old = tc.mem;  // forgotten before the free is checked
                            tc.mem = nullptr;
                            tc.bytes = 0;
                            HIPCHK(h, hipFree(old));
                        }
                        if (hipMalloc(&tc.mem, tc_bytes) != hipSuccess) {
                            tc.mem = nullptr;
                            set_err(h, "hipMalloc of %zu bytes for the table cache failed",
                                    tc_bytes);
                            throw Fail{PHOEBE_E_NOMEM};
                        }
                        tc.bytes = tc_bytes;
                    }
                    size_t o = 0;
                    for (int i = 0; i < 5; ++i) {
                        HIPCHK(h, hipMemcpyAsync(tc.mem + o, parts[i], sizes[i],
                                                 hipMemcpyDeviceToDevice, s));
                        o += sizes[i];
                    }
                    tc.h_r = sys->h_r;
                    tc.phi_r = sys->phi_r;
                    tc.mass = sys->mass;
                    tc.rh = rh_v;
                    tc.rd = rd_v;
                    tc.nW = nW;
                    tc.nat = sys->n_atoms;
                    tc.n0 = mesh.n0;
                    tc.n1 = mesh.n1;
                    tc.n2 = mesh.n2;
                    tc.omega_min = par->omega_min;
                    tc.kT = par->kT;
                    tc.valid = true;
                }
            }
        }
        HIPCHK(h, launch_fermi(T.eps, N * nW, par->mu, par->kT, T.focc, s));
        HIPCHK(h, launch_band_extrema(T.eps, N, nW, T.omega, N, nm, T.bmin, T.bmax, T.wmax, s));
        HIPCHK(h, launch_window(T.eps, N, nW, par->win_lo, par->win_hi, T.mask, T.flag, s));
        if (polar) {
            HIPCHK(h, hipMemcpyAsync(T.born, sys->polar->born, sizeof(double) * 9 * sys->n_atoms,
                                     hipMemcpyHostToDevice, s));
            HIPCHK(h, launch_polar_factor(nullptr, mesh, N, T.E, nm, polar_dev(sys, T.born), T.Lpol, s));
        }
        // adaptive smearing: velocities on the mesh; the widest width any transition
        // can take bounds the final-band pruning
        double sigma_bound = par->sigma;
        const double ad_pref = adaptive ? par->adaptive_scale / std::sqrt(12.0) : 0.0;
        const double ad_c[3] = {ad_pref * 2.0 * kPi / mesh.n0, ad_pref * 2.0 * kPi / mesh.n1,
                                ad_pref * 2.0 * kPi / mesh.n2};
        if (adaptive) {
            Arena b3 = ar;
            velocity_dev(h, b3, sys, T.rh, nullptr, mesh, N, T.eps, T.U, true, T.vel, T.vbad, s);
            HIPCHK(h, launch_velocity_max(T.vel, N, nW, T.vmax, s));
            double vm[3];
            int32_t bad = 0;
            HIPCHK(h, hipMemcpyAsync(vm, T.vmax, sizeof vm, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipMemcpyAsync(&bad, T.vbad, sizeof bad, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            if (bad) {
                set_err(h, "a degenerate group of more than 8 bands in the velocity operator");
                throw Fail{PHOEBE_E_UNSUPPORTED};
            }
            double s2 = 0.0;
            for (int d = 0; d < 3; ++d) s2 += (ad_c[d] * 2.0 * vm[d]) * (ad_c[d] * 2.0 * vm[d]);
            sigma_bound = std::max(par->sigma, std::sqrt(s2));
        }
        if (lw_out) {
            HIPCHK(h, launch_zero(T.lwacc, sizeof(double) * N * nm, s));
            HIPCHK(h, launch_zero(lw_out, sizeof(double) * N * nm, s));
        }
        int64_t rows = nk;
        const int32_t* kept = k_idx;
        if (!k_idx) {
            HIPCHK(h, launch_compact(T.flag, N, T.kept, T.cnt, s));
            int32_t c = 0;
            HIPCHK(h, hipMemcpyAsync(&c, T.cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            rows = c;
            kept = T.kept;
        } else {
            std::vector<int32_t> kh(nk);
            HIPCHK(h, hipMemcpyAsync(kh.data(), k_idx, sizeof(int32_t) * nk, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            for (int64_t i = 0; i < nk; ++i)
                REQUIRE(h, kh[i] >= 0 && kh[i] < N, "k_idx[%lld] = %d is not a mesh index",
                        (long long)i, kh[i]);
        }
        if (n_kept_out) *n_kept_out = rows;
        HIPCHK(h, launch_zero(gamma_out, (size_t)rows * nW * sizeof(double), s));
        if (rows == 0) return;
        HIPCHK(h, launch_gather_rows(T.mask, kept, rows, nW, T.rowflag, band_mask, kept_k_out, s));
        HIPCHK(h, launch_compact(T.rowflag, rows * nW, T.ids, T.cnt + 1, s));
        int32_t nst_i = 0;
        HIPCHK(h, hipMemcpyAsync(&nst_i, T.cnt + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        const int nst = nst_i;
        if (n_states_out) *n_states_out = nst;
        REQUIRE(h, state_cap < 0 || nst <= state_cap,
                "%d states in the window exceed the per-state output capacity of %lld", nst,
                (long long)state_cap);
        if (nst == 0) {
            flush_timing(h, s);
            return;
        }
        const double cut = 27.5 * sigma_bound;  // exp(-27.5^2) underflows to 0 in FP64
        HIPCHK(h, launch_build_states(T.ids, nst, nW, kept, T.eps, T.bmin, T.bmax, T.wmax, cut,
                                      T.st_row, T.st_band, T.st_kmesh, T.st_mlo, T.st_mhi, s));
        if (dweights)
            HIPCHK(h, launch_delta_weights(nst, N, mesh, T.st_kmesh, T.st_band, T.st_mlo, T.st_mhi,
                                           T.eps, T.focc, T.omega, T.nb, nW, nm, par->sigma,
                                           par->omega_min,
                                           2.0 * kPi / (std::sqrt(kPi) * par->sigma), dweights, s));
        if (terms || dweights) {
            if (terms) HIPCHK(h, launch_zero(terms, (size_t)nst * N * nm * sizeof(double), s));
            if (st_row_out)
                HIPCHK(h, hipMemcpyAsync(st_row_out, T.st_row, 4 * (size_t)nst, hipMemcpyDeviceToDevice, s));
            if (st_band_out)
                HIPCHK(h, hipMemcpyAsync(st_band_out, T.st_band, 4 * (size_t)nst, hipMemcpyDeviceToDevice, s));
        }
        if (!rates) {
            HIPCHK(h, hipStreamSynchronize(s));
            flush_timing(h, s);
            return;
        }
        std::vector<int32_t> strow(nst);
        HIPCHK(h, hipMemcpyAsync(strow.data(), T.st_row, sizeof(int32_t) * nst,
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));

        // ---- phase B: batches of kept-k rows ----
        // Direct stage 1: BK rows each.  Factorised stage 1: consecutive rows
        // while the batch holds at most BK rows, kD0Max distinct k0 and kD01Max
        // distinct (k0, k1), with the grouping lists the axis kernels use.
        std::vector<std::pair<int64_t, int64_t>> batches;
        std::vector<int32_t> rbh;          // grouping lists of every batch, one array
        std::vector<std::array<int64_t, 11>> rbo;  // per batch: d0, d01, offsets of the 8 lists
        std::vector<int32_t> planes;               // every distinct k0 of the call, ascending
        if (!re_fact) {
            for (int64_t r0 = 0; r0 < rows; r0 += BK) batches.push_back({r0, std::min<int64_t>(BK, rows - r0)});
        } else {
            std::vector<int32_t> kh(rows);
            HIPCHK(h, hipMemcpyAsync(kh.data(), kept, sizeof(int32_t) * rows, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            const int64_t n12 = (int64_t)mesh.n1 * mesh.n2;
            if (all_planes) {
                for (int64_t i = 0; i < rows; ++i) planes.push_back((int32_t)(kh[i] / n12));
                std::sort(planes.begin(), planes.end());
                planes.erase(std::unique(planes.begin(), planes.end()), planes.end());
            }
            int64_t r = 0;
            while (r < rows) {
                std::vector<int32_t> k0s, prs;  // distinct k0 and pair ids k0 n1 + k1
                int64_t e = r;
                while (e < rows && e - r < BK) {
                    const int32_t k0 = (int32_t)(kh[e] / n12);
                    const int32_t pr = (int32_t)(kh[e] / mesh.n2);
                    const bool n0 = std::find(k0s.begin(), k0s.end(), k0) == k0s.end();
                    const bool n01 = std::find(prs.begin(), prs.end(), pr) == prs.end();
                    if ((!all_planes && (int)k0s.size() + n0 > kD0Max) ||
                        (int)prs.size() + n01 > kD01Max)
                        break;
                    if (n0) k0s.push_back(k0);
                    if (n01) prs.push_back(pr);
                    ++e;
                }
                std::sort(k0s.begin(), k0s.end());
                std::sort(prs.begin(), prs.end());
                const int d0 = (int)k0s.size(), d01 = (int)prs.size();
                const int64_t nb = e - r;
                std::array<int64_t, 11> o{};
                o[0] = d0;
                o[1] = d01;
                // d_k0
                o[2] = (int64_t)rbh.size();
                rbh.insert(rbh.end(), k0s.begin(), k0s.end());
                // pair_k1 and pair_off (pairs are sorted by k0, then k1)
                o[3] = (int64_t)rbh.size();
                for (int32_t pr : prs) rbh.push_back(pr % mesh.n1);
                o[4] = (int64_t)rbh.size();
                {
                    int pp = 0;
                    for (int d = 0; d <= d0; ++d) {
                        while (d < d0 && pp < d01 && prs[pp] / mesh.n1 < k0s[d]) ++pp;
                        rbh.push_back(pp);
                    }
                    rbh[o[4] + d0] = d01;
                }
                // rows grouped by pair: kp_off, k_row (batch-local), k_k2
                std::vector<std::vector<int32_t>> byp(d01);
                for (int64_t i = r; i < e; ++i) {
                    const int32_t pr = (int32_t)(kh[i] / mesh.n2);
                    const int pidx = (int)(std::lower_bound(prs.begin(), prs.end(), pr) - prs.begin());
                    byp[pidx].push_back((int32_t)(i - r));
                }
                o[5] = (int64_t)rbh.size();
                {
                    int32_t acc = 0;
                    for (int pp = 0; pp < d01; ++pp) {
                        rbh.push_back(acc);
                        acc += (int32_t)byp[pp].size();
                    }
                    rbh.push_back(acc);
                }
                o[6] = (int64_t)rbh.size();
                for (int pp = 0; pp < d01; ++pp) rbh.insert(rbh.end(), byp[pp].begin(), byp[pp].end());
                o[7] = (int64_t)rbh.size();
                for (int pp = 0; pp < d01; ++pp)
                    for (int32_t lr : byp[pp]) rbh.push_back((int32_t)(kh[r + lr] % mesh.n2));
                // d_plane: position of each distinct k0 in the call's plane list
                o[8] = (int64_t)rbh.size();
                for (int32_t k0 : k0s)
                    rbh.push_back(all_planes ? (int32_t)(std::lower_bound(planes.begin(), planes.end(),
                                                                           k0) - planes.begin())
                                             : 0);
                // row_st: first state (batch-local) of every batch row, and the end
                o[9] = (int64_t)rbh.size();
                std::vector<int32_t> rst(nb + 1);
                {
                    const int64_t s0 = std::lower_bound(strow.begin(), strow.end(), (int32_t)r) -
                                       strow.begin();
                    for (int64_t i = r; i <= e; ++i)
                        rst[i - r] = (int32_t)(std::lower_bound(strow.begin(), strow.end(),
                                                                (int32_t)i) - strow.begin() - s0);
                    rbh.insert(rbh.end(), rst.begin(), rst.end());
                }
                // k_ent: per entry of k_row, (k2, first state, end of states, 0), 16-byte aligned
                while (rbh.size() % 4) rbh.push_back(0);
                o[10] = (int64_t)rbh.size();
                for (int pp = 0; pp < d01; ++pp)
                    for (int32_t lr : byp[pp]) {
                        rbh.push_back((int32_t)(kh[r + lr] % mesh.n2));
                        rbh.push_back(rst[lr]);
                        rbh.push_back(rst[lr + 1]);
                        rbh.push_back(0);
                    }
                rbo.push_back(o);
                batches.push_back({r, nb});
                r = e;
            }
            if (all_planes) {  // the plane list itself, after the batch lists
                rbo.push_back({(int64_t)planes.size(), 0, (int64_t)rbh.size(), 0, 0, 0, 0, 0, 0, 0, 0});
                rbh.insert(rbh.end(), planes.begin(), planes.end());
            }
            REQUIRE(h, rbh.size() <= (size_t)rows_cap * 176, "stage-1 grouping lists too long");
        }
        int32_t* rbd = re_fact ? ar.take<int32_t>(std::max<size_t>(rbh.size(), 1)) : nullptr;
        if (re_fact)
            HIPCHK(h, hipMemcpyAsync(rbd, rbh.data(), sizeof(int32_t) * rbh.size(),
                                     hipMemcpyHostToDevice, s));
        char* T0re = re_fact ? ar.take<char>(t0_bytes) : nullptr;
        cd* P1 = ar.take<cd>((size_t)BK * n_re);
        char* Gbuf = fold_fused ? nullptr : ar.take<char>((size_t)BK * NC2 * g_elem);
        char* Fbuf = ar.take<char>((size_t)max_states * rp_pad * nc_pad * f_elem);
        double* partial = ar.take<double>((size_t)max_states * n_qtiles);
        char* T1buf = factored && !axes_fused
                          ? ar.take<char>((size_t)nsb * Wbox * Wbox * mesh.n2 * nc_pad * g_elem)
                          : nullptr;
        char* T2buf = factored ? ar.take<char>((size_t)nsb * Wbox * NL * nc_pad * g_elem) : nullptr;
        uint32_t* livebuf = factored ? ar.take<uint32_t>((size_t)nsb * NL * n0_line) : nullptr;
        uint32_t* lineany = factored ? ar.take<uint32_t>((size_t)nsb * NL) : nullptr;
        double* lwbuf = lw_out ? ar.take<double>((factored ? (size_t)nsb * NL * n0_line
                                                           : (size_t)max_states * N) * nm)
                               : nullptr;
        // live (state, line) count of every factorised sub-batch (traffic accounting)
        int64_t n_sub = 0;
        if (factored)
            for (const auto& bt : batches) {
                const int64_t a0 = std::lower_bound(strow.begin(), strow.end(), (int32_t)bt.first) -
                                   strow.begin();
                const int64_t a1 = std::lower_bound(strow.begin(), strow.end(),
                                                    (int32_t)(bt.first + bt.second)) - strow.begin();
                n_sub += (a1 - a0 + nsb - 1) / nsb;
            }
        uint32_t* nlive = factored ? ar.take<uint32_t>((size_t)2 * std::max<int64_t>(n_sub, 1)) : nullptr;
        if (factored)
            HIPCHK(h, hipMemsetAsync(nlive, 0, 2 * sizeof(uint32_t) * std::max<int64_t>(n_sub, 1), s));
        int64_t isub = 0;

        // adaptive: every term carries its own 1/sigma_t, so the common factor has sigma = 1
        const double inv_sqrtpi_sigma = 1.0 / (std::sqrt(kPi) * (adaptive ? 1.0 : par->sigma));
        const double scale = 2.0 * kPi * inv_sqrtpi_sigma * (q_off ? 1.0 : 1.0 / (double)N);
        if (fold_fused)  // F's padding (rows >= n_rp, columns of no mode) is never written
            HIPCHK(h, launch_zero_fpad(Fbuf, max_states, rp_pad, nc_pad, n_rp, 16 * nm, (int)f_elem,
                                       s));
        if (all_planes) {
            // T0 of every k0 plane of the call: g(Re,Rp) read once, the planes written once
            const auto& o = rbo.back();
            Timer tp(h, s, "stage1_planes");
            if (lowp)
                HIPCHK(h, launch_re_planes_f32(reinterpret_cast<const cd*>(sys->g_rr), NC2, T.box_re,
                                               rmax_e, T.Pre, rbd + o[2], (int)o[0], fold_fused,
                                               reinterpret_cast<cf*>(T0re), s));
            else
                HIPCHK(h, launch_re_planes(reinterpret_cast<const cd*>(sys->g_rr), NC2, T.box_re,
                                           rmax_e, T.Pre, rbd + o[2], (int)o[0], fold_fused,
                                           reinterpret_cast<cd*>(T0re), s));
            tp.done((double)NC2 * (16.0 * n_re + (double)g_elem * (double)o[0] * We * We));
        }
        int sbeg = 0;
        for (size_t bi = 0; bi < batches.size(); ++bi) {
            const int64_t r0 = batches[bi].first, nb = batches[bi].second;
            int send = sbeg;
            while (send < nst && strow[send] < r0 + nb) ++send;
            const int ns = send - sbeg;
            if (ns == 0) continue;
            if (re_fact) {
                const auto& o = rbo[bi];
                ReBatch rb{(int)o[0], (int)o[1], rbd + o[2], rbd + o[3], rbd + o[4],
                           rbd + o[5], rbd + o[6], rbd + o[7], all_planes ? rbd + o[8] : nullptr,
                           rbd + o[10]};
                FoldOut fo{rbd + o[9], T.st_kmesh + sbeg, T.st_band + sbeg, T.U,
                           nW, nm, n_rp, rp_pad, nc_pad, Fbuf};
                const FoldOut* fop = fold_fused ? &fo : nullptr;
                // written once: G, or F when the fold is applied here
                const double out_bytes = fold_fused ? (double)ns * n_rp * nm * nW * f_elem
                                                    : (double)nb * NC2 * g_elem;
                Timer t1(h, s, "stage1_axes");
                if (all_planes) {
                    if (lowp)
                        HIPCHK(h, launch_re_pairs_f32(reinterpret_cast<const cf*>(T0re), NC2, rmax_e,
                                                      mesh, T.Pre, rb, fop,
                                                      reinterpret_cast<cf*>(Gbuf), NC2, s));
                    else
                        HIPCHK(h, launch_re_pairs(reinterpret_cast<const cd*>(T0re), NC2, rmax_e, mesh,
                                                  T.Pre, rb, fop, reinterpret_cast<cd*>(Gbuf), NC2, s));
                    // the batch's T0 planes read once
                    t1.done((double)NC2 * (double)g_elem * rb.d0 * We * We + out_bytes);
                } else {
                    if (lowp)
                        HIPCHK(h, launch_re_axes_f32(reinterpret_cast<const cd*>(sys->g_rr), NC2,
                                                     T.box_re, rmax_e, mesh, T.Pre, rb, fop,
                                                     reinterpret_cast<cf*>(T0re),
                                                     reinterpret_cast<cf*>(Gbuf), NC2, s));
                    else
                        HIPCHK(h, launch_re_axes(reinterpret_cast<const cd*>(sys->g_rr), NC2,
                                                 T.box_re, rmax_e, mesh, T.Pre, rb, fop,
                                                 reinterpret_cast<cd*>(T0re),
                                                 reinterpret_cast<cd*>(Gbuf), NC2, s));
                    // g (FP64) read once; T0 written and read once
                    t1.done((double)NC2 * (16.0 * n_re + (double)g_elem * 2.0 * rb.d0 * We * We) +
                            out_bytes);
                }
            } else {
            HIPCHK(h, launch_phase_table(nullptr, kept + r0, mesh, nb, T.re, n_re, P1, n_re, s));
            Timer t1(h, s, "stage1_phase");
            if (lowp)
                HIPCHK(h, launch_cgemm_lp(prec, P1, n_re, reinterpret_cast<const cd*>(sys->g_rr), NC2,
                                          reinterpret_cast<cf*>(Gbuf), NC2, nb, NC2, n_re, s));
            else
                HIPCHK(h, launch_zgemm(P1, n_re, reinterpret_cast<const cd*>(sys->g_rr), NC2,
                                       reinterpret_cast<cd*>(Gbuf), NC2, nb, NC2, n_re, s));
            t1.done();
            }
            if (fold_fused) {
                // F written by the stage-1 pair and k kernel
            } else if (lowp)
                HIPCHK(h, launch_fold_uk_lp(prec, reinterpret_cast<const cf*>(Gbuf), NC2, T.U,
                                            T.st_row + sbeg, (int)r0, T.st_kmesh + sbeg,
                                            T.st_band + sbeg, ns, n_rp, nm, nW, cw, rp_pad, nc_pad,
                                            Fbuf, s));
            else
                HIPCHK(h, launch_fold_uk(reinterpret_cast<const cd*>(Gbuf), NC2, T.U, T.st_row + sbeg,
                                         (int)r0, T.st_kmesh + sbeg, T.st_band + sbeg, ns, n_rp, nm,
                                         nW, cw, rp_pad, nc_pad, reinterpret_cast<cd*>(Fbuf), s));
            RateArgs ra{};
            ra.F = reinterpret_cast<const cd*>(Fbuf);
            ra.rp_pad = rp_pad;
            ra.nc_pad = nc_pad;
            ra.n_rp = n_rp;
            ra.rp_packed = T.rp_packed;
            ra.rmax = rmax_p;
            ra.mesh = mesh;
            ra.nq_mesh = N;
            ra.st_kmesh = T.st_kmesh + sbeg;
            ra.st_band = T.st_band + sbeg;
            ra.st_row = T.st_row + sbeg;
            ra.st_mlo = T.st_mlo + sbeg;
            ra.st_mhi = T.st_mhi + sbeg;
            ra.q_off = q_off;
            ra.q_idx = q_idx;
            ra.q_w = q_w;
            ra.eps = T.eps;
            ra.focc = T.focc;
            ra.U = T.U;
            ra.omega = T.omega;
            ra.nb = T.nb;
            ra.E = T.E;
            ra.nW = nW;
            ra.nm = nm;
            ra.sigma = par->sigma;
            ra.partial = partial;
            ra.n_qtiles = n_qtiles;
            ra.terms = terms ? terms + (int64_t)sbeg * N * nm : nullptr;
            ra.terms_scale = 2.0 * kPi * inv_sqrtpi_sigma;
            ra.Lpol = polar ? T.Lpol : nullptr;
            ra.vel = adaptive ? T.vel : nullptr;
            for (int d = 0; d < 3; ++d) ra.ad_c[d] = ad_c[d];
            ra.lw = lwbuf;
            ra.inv_kT = 1.0 / par->kT;
            if (lowp && !factored) {
                Timer t2(h, s, "stage2_rates");
                RateArgsLP rl{};
                rl.F = Fbuf;
                rl.rp_pad = ra.rp_pad; rl.nc_pad = ra.nc_pad; rl.n_rp = ra.n_rp;
                rl.rp_packed = ra.rp_packed; rl.rmax = ra.rmax; rl.mesh = ra.mesh;
                rl.nq_mesh = ra.nq_mesh; rl.st_kmesh = ra.st_kmesh; rl.st_band = ra.st_band;
                rl.st_row = ra.st_row; rl.st_mlo = ra.st_mlo; rl.st_mhi = ra.st_mhi;
                rl.q_off = ra.q_off; rl.q_idx = ra.q_idx; rl.q_w = ra.q_w; rl.eps = ra.eps;
                rl.focc = ra.focc; rl.U = ra.U; rl.omega = ra.omega; rl.nb = ra.nb; rl.E = ra.E;
                rl.nW = nW; rl.nm = nm; rl.sigma = ra.sigma; rl.partial = partial;
                rl.n_qtiles = n_qtiles;
                HIPCHK(h, launch_stage2_rates_lp(prec, rl, ns, s));
                t2.done();
            } else if (!factored) {
                if (lwbuf) HIPCHK(h, launch_zero(lwbuf, sizeof(double) * ns * N * nm, s));
                Timer t2(h, s, "stage2_rates");
                HIPCHK(h, launch_stage2_rates(ra, ns, s));
                t2.done();
                if (lwbuf) HIPCHK(h, launch_lw_reduce_dense(lwbuf, ns, N, nm, T.lwacc, s));
            } else {
                ra.P0 = T.Pax;
                ra.W = Wbox;
                ra.wmax = T.wmax;
                for (int sb = 0; sb < ns; sb += nsb) {
                    const int nn = std::min(nsb, ns - sb);
                    REQUIRE(h, isub < n_sub, "sub-batch count");
                    uint32_t* nl = nlive + 2 * isub++;
                    RateArgs rb = ra;
                    rb.T2 = T2buf;
                    rb.st_kmesh += sb;
                    rb.st_band += sb;
                    rb.st_row += sb;
                    rb.st_mlo += sb;
                    rb.st_mhi += sb;
                    rb.partial = partial + (int64_t)sb * n_qtiles;
                    if (ra.terms) rb.terms = ra.terms + (int64_t)sb * N * nm;
                    rb.live = livebuf;
                    rb.line_bands = lineany;
                    // live bands of every (state, line, chunk) first: T2 is formed for live lines only
                    HIPCHK(h, launch_line_live(rb, nn, livebuf, lineany, nl, s));
                    Timer ta(h, s, "axis_transforms");
                    if (lowp)
                        HIPCHK(h, launch_axis_transforms_f32(
                                      reinterpret_cast<const cf*>(Fbuf) + (int64_t)sb * rp_pad * nc_pad,
                                      rp_pad, nc_pad, T.box_rp, rmax_p, mesh, T.Pax, nn, lineany,
                                      reinterpret_cast<cf*>(T1buf), reinterpret_cast<cf*>(T2buf), s));
                    else
                        HIPCHK(h, launch_axis_transforms(
                                      reinterpret_cast<const cd*>(Fbuf) + (int64_t)sb * rp_pad * nc_pad,
                                      rp_pad, nc_pad, T.box_rp, rmax_p, mesh, T.Pax, nn, lineany,
                                      reinterpret_cast<cd*>(T1buf), reinterpret_cast<cd*>(T2buf), s));
                    // F read once, T2 written for the live lines; T1 written and read once
                    // unless both axes ran in one pass
                    const double ab = (double)g_elem * nm * nW;
                    const double t1_rw = axis_transforms_fused(rmax_p, nc_pad, lowp)
                                             ? 0.0
                                             : 2.0 * Wbox * Wbox * mesh.n2;
                    ta.done(ab * nn * ((double)n_rp + t1_rw), nl, ab * Wbox);
                    Timer tl(h, s, "line_rates");
                    if (lowp)
                        HIPCHK(h, launch_line_rates_f32(rb, nn, s));
                    else
                        HIPCHK(h, launch_line_rates(rb, nn, s));
                    // T2 of every live (state, line) read once; U_{k+q} of band m at the 16
                    // points of every unit
                    tl.done(0.0, nl, (double)g_elem * Wbox * nm * nW, nl + 1, 16.0 * nW * sizeof(cd));
                    if (lwbuf)
                        HIPCHK(h, launch_lw_reduce_lines(lwbuf, lineany, livebuf, nn, (int)NL,
                                                         mesh.n0, nm, T.lwacc, s));
                }
            }
            HIPCHK(h, launch_reduce_partials(partial, ns, n_qtiles, T.st_row + sbeg,
                                             T.st_band + sbeg, nW, scale, gamma_out, s));
            sbeg = send;
        }
        if (lw_out)  // (2 pi / N_k) n (n + 1) hbar omega x the sums, with the delta's 1/(sqrt(pi) sigma)
            HIPCHK(h, launch_lw_finish(T.lwacc, T.omega, T.nb, N * nm, par->omega_min,
                                       2.0 * kPi * inv_sqrtpi_sigma / (double)N, lw_out, s));
        HIPCHK(h, hipGetLastError());
        flush_timing(h, s);
    });
}

extern "C" {

phoebe_status phoebe_gpu_scatter_rates(void* handle, const phoebe_system* sys,
                                       const int32_t k_mesh[3], const int32_t q_mesh[3],
                                       const int32_t* k_idx, int64_t nk,
                                       const int64_t* q_off, const int32_t* q_idx,
                                       const double* q_w, const phoebe_rate_params* par,
                                       phoebe_precision prec, double* gamma_out,
                                       uint8_t* band_mask, int32_t* kept_k_out,
                                       int64_t* n_kept_out, void* stream) {
    if (handle && !q_mesh) {
        static_cast<Handle*>(handle)->err = "q_mesh is NULL";
        return PHOEBE_E_INVALID;
    }
    return scatter_rates_impl(handle, sys, k_mesh, q_mesh, nullptr, k_idx, nk, q_off, q_idx, q_w,
                              par, prec, gamma_out, band_mask, kept_k_out, n_kept_out, nullptr,
                              nullptr, nullptr, nullptr, nullptr, true, -1, stream);
}

phoebe_status phoebe_gpu_phonon_linewidth(void* handle, const phoebe_system* sys,
                                          const int32_t k_mesh[3], const int32_t q_mesh[3],
                                          const phoebe_rate_params* par, phoebe_precision prec,
                                          double* p_out, double* gamma_out, int64_t* n_kept_out,
                                          void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    if (!p_out || !q_mesh || !k_mesh) {
        h->err = "p_out, k_mesh or q_mesh is NULL";
        return PHOEBE_E_INVALID;
    }
    if (prec != PHOEBE_FP64) {
        h->err = "the phonon linewidth is computed in FP64 only";
        return prec >= PHOEBE_FP64 && prec <= PHOEBE_BF16 ? PHOEBE_E_UNSUPPORTED : PHOEBE_E_INVALID;
    }
    // the electron rates of the same pass go to gamma_out, or to workspace rows
    double* g = gamma_out;
    bool own = false;
    if (!g) {
        if (k_mesh[0] < 1 || k_mesh[1] < 1 || k_mesh[2] < 1) {
            h->err = "mesh must be >= 1";
            return PHOEBE_E_INVALID;
        }
        const size_t rows = (size_t)k_mesh[0] * k_mesh[1] * k_mesh[2];
        if (sys && sys->n_wannier >= 1 && sys->n_wannier <= 64 && rows <= ((size_t)1 << 30)) {
            if (hipMalloc(reinterpret_cast<void**>(&g), rows * sys->n_wannier * sizeof(double)) !=
                hipSuccess) {
                h->err = "hipMalloc of the rate rows failed";
                return PHOEBE_E_NOMEM;
            }
            own = true;
        }
    }
    const phoebe_status st = scatter_rates_impl(handle, sys, k_mesh, q_mesh, p_out, nullptr, 0,
                                                nullptr, nullptr, nullptr, par, prec, g, nullptr,
                                                nullptr, n_kept_out, nullptr, nullptr, nullptr,
                                                nullptr, nullptr, true, -1, stream);
    if (own) {
        (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
        (void)hipFree(g);
    }
    return st;
}

phoebe_status phoebe_gpu_set_fault_injection(void* handle, int64_t at) {
    if (!handle || at < 0) return PHOEBE_E_INVALID;
    static_cast<Handle*>(handle)->inject_at = at;
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_set_table_cache(void* handle, int enable) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    h->table_cache = enable != 0;
    h->tc.valid = false;  // on or off, the next call builds its tables
    if (!enable && h->tc.mem) {
        (void)hipSetDevice(h->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(h->tc.mem);
        h->tc.mem = nullptr;
        h->tc.bytes = 0;
    }
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_set_check_finite(void* handle, int enable) {
    if (!handle) return PHOEBE_E_INVALID;
    static_cast<Handle*>(handle)->check_finite = enable != 0;
    return PHOEBE_OK;
}

phoebe_status phoebe_gpu_velocities(void* handle, const phoebe_system* sys, const double* k_frac,
                                    int64_t nk, double* eps_out, double* v_out, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        check_system(h, sys, true, false, false);
        REQUIRE(h, nk >= 0, "nk < 0");
        if (nk == 0) return;
        REQUIRE(h, k_frac && v_out, "k_frac/v_out is NULL");
        REQUIRE(h, sys->n_wannier <= 32, "n_wannier > 32 is not supported");
        HIPCHK(h, hipSetDevice(h->device));
        scan_finite(h, sys, true, false, false, s);
        const int nW = sys->n_wannier;
        auto plan = [&](Arena& ar) {
            int32_t* rh = upload_r(h, ar, sys->rh, sys->n_rh, s);
            double* eps = eps_out ? eps_out : ar.take<double>((size_t)nk * nW);
            cd* U = ar.take<cd>((size_t)nk * nW * nW);
            int32_t* bad = ar.take<int32_t>(1);
            Arena a1 = ar, a2 = ar;
            electron_bands_dev(h, a1, sys, rh, k_frac, nullptr, Mesh{1, 1, 1}, nk, eps, U, s);
            velocity_dev(h, a2, sys, rh, k_frac, Mesh{1, 1, 1}, nk, eps, U, false, v_out, bad, s);
            ar.used = std::max(a1.used, a2.used);
            if (!ar.base) return;
            int32_t b = 0;
            HIPCHK(h, hipMemcpyAsync(&b, bad, sizeof b, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            if (b) {
                set_err(h, "a degenerate group of more than 8 bands in the velocity operator");
                throw Fail{PHOEBE_E_UNSUPPORTED};
            }
        };
        Arena dry(nullptr);
        plan(dry);
        ensure_ws(h, dry.used);
        Arena ar(h->ws, h->ws_cap);
        plan(ar);
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipStreamSynchronize(s));
        flush_timing(h, s);
    });
}

phoebe_status phoebe_gpu_polar_factor(void* handle, const phoebe_system* sys, const double* q_frac,
                                      int64_t nq, double omega_min, phoebe_c128* l_out,
                                      void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        check_system(h, sys, false, true, false);
        REQUIRE(h, sys->polar != nullptr, "the system has no polar data");
        check_polar(h, sys);
        REQUIRE(h, nq >= 0, "nq < 0");
        REQUIRE(h, std::isfinite(omega_min) && omega_min >= 0.0, "omega_min must be >= 0");
        if (nq == 0) return;
        REQUIRE(h, q_frac && l_out, "q_frac/l_out is NULL");
        HIPCHK(h, hipSetDevice(h->device));
        scan_finite(h, sys, false, true, false, s);
        const int nm = 3 * sys->n_atoms;
        auto plan = [&](Arena& ar) {
            int32_t* rd = upload_r(h, ar, sys->rd, sys->n_rd, s);
            double* born = ar.take<double>((size_t)9 * sys->n_atoms);
            double* om = ar.take<double>((size_t)nq * nm);
            cd* E = ar.take<cd>((size_t)nq * nm * nm);
            phonon_dev(h, ar, sys, rd, q_frac, nullptr, Mesh{1, 1, 1}, nq, omega_min, 0.0, om, E,
                       nullptr, nullptr, s);
            if (!ar.base) return;
            HIPCHK(h, hipMemcpyAsync(born, sys->polar->born, sizeof(double) * 9 * sys->n_atoms,
                                     hipMemcpyHostToDevice, s));
            HIPCHK(h, launch_polar_factor(q_frac, Mesh{1, 1, 1}, nq, E, nm, polar_dev(sys, born),
                                          reinterpret_cast<cd*>(l_out), s));
        };
        Arena dry(nullptr);
        plan(dry);
        ensure_ws(h, dry.used);
        Arena ar(h->ws, h->ws_cap);
        plan(ar);
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipStreamSynchronize(s));
    });
}

phoebe_status phoebe_gpu_rate_terms(void* handle, const phoebe_system* sys, const int32_t mesh[3],
                                    const int32_t* k_idx, int64_t nk,
                                    const phoebe_rate_params* par, double* gamma_out,
                                    double* terms, double* dweights, int32_t* st_row,
                                    int32_t* st_band, int64_t max_states, int64_t* n_states,
                                    void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    if (!terms) {
        static_cast<Handle*>(handle)->err = "terms is NULL";
        return PHOEBE_E_INVALID;
    }
    return scatter_rates_impl(handle, sys, mesh, nullptr, nullptr, k_idx, nk, nullptr, nullptr,
                              nullptr, par, PHOEBE_FP64, gamma_out, nullptr, nullptr, nullptr, terms,
                              st_row, st_band, n_states, dweights, true, max_states, stream);
}

phoebe_status phoebe_gpu_delta_weights(void* handle, const phoebe_system* sys,
                                       const int32_t mesh[3], const int32_t* k_idx, int64_t nk,
                                       const phoebe_rate_params* par, double* dweights,
                                       int32_t* st_row, int32_t* st_band, int64_t max_states,
                                       int64_t* n_states, double* gamma_scratch, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    if (!dweights) {
        static_cast<Handle*>(handle)->err = "dweights is NULL";
        return PHOEBE_E_INVALID;
    }
    return scatter_rates_impl(handle, sys, mesh, nullptr, nullptr, k_idx, nk, nullptr, nullptr,
                              nullptr, par, PHOEBE_FP64, gamma_scratch, nullptr, nullptr, nullptr,
                              nullptr, st_row, st_band, n_states, dweights, false, max_states,
                              stream);
}

}  // extern "C"
