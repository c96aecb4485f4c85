// C ABI of the 3-phonon coupling interpolation, the Philox streams, the
// network initialisation, the training-set builder and the row gather.
#include "host.hpp"

using namespace phx;

extern "C" {

phoebe_status phoebe_gpu_interp_v3(void* handle, const phoebe_system3* sys, const double* q_frac,
                                   int64_t nq, const double* qp_frac, int64_t nqp,
                                   double omega_min, phoebe_c128* v3_out, double* omega_q,
                                   double* omega_qp, double* omega_qpp, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        REQUIRE(h, sys != nullptr, "system is NULL");
        REQUIRE(h, sys->n_atoms >= 1, "n_atoms must be >= 1");
        REQUIRE(h, sys->n_rd >= 1 && sys->rd && sys->phi_r && sys->mass, "force constants missing");
        REQUIRE(h, sys->n_r1 >= 1 && sys->r1 && sys->n_r2 >= 1 && sys->r2 && sys->phi3,
                "third-order constants missing");
        REQUIRE(h, nq >= 0 && nqp >= 0, "negative nq or nqp");
        REQUIRE(h, std::isfinite(omega_min) && omega_min >= 0.0, "omega_min must be >= 0");
        if (nq == 0 || nqp == 0) return;
        REQUIRE(h, q_frac && qp_frac && v3_out, "q_frac/qp_frac/v3_out is NULL");
        if (sys->n_atoms > 10) {
            set_err(h, "more than 10 atoms (30 modes) is not supported");
            throw Fail{PHOEBE_E_UNSUPPORTED};
        }
        REQUIRE(h, nq * nqp <= 1000000, "nq * nqp above 1e6 pairs: split the call");
        HIPCHK(h, hipSetDevice(h->device));
        const int nm = 3 * sys->n_atoms;
        const int64_t m3 = (int64_t)nm * nm * nm;
        const int n1 = sys->n_r1, n2 = sys->n_r2;
        // the harmonic part as a phoebe_system for the phonon solver
        phoebe_system ph{};
        ph.n_wannier = 1;
        ph.n_atoms = sys->n_atoms;
        ph.n_rd = sys->n_rd;
        ph.rd = sys->rd;
        ph.phi_r = sys->phi_r;
        ph.mass = sys->mass;
        // e^{-i 2 pi q.R}: phase tables of the negated lattice vectors
        std::vector<int32_t> nr1(3 * (size_t)n1), nr2(3 * (size_t)n2);
        for (int i = 0; i < 3 * n1; ++i) nr1[i] = -sys->r1[i];
        for (int i = 0; i < 3 * n2; ++i) nr2[i] = -sys->r2[i];
        const int64_t qb = std::min<int64_t>(nq, 16);  // q of one stage-1 batch
        auto plan = [&](Arena& ar) {
            int32_t* rd = upload_r(h, ar, sys->rd, sys->n_rd, s);
            int32_t* r1 = upload_r(h, ar, nr1.data(), n1, s);
            int32_t* r2 = upload_r(h, ar, nr2.data(), n2, s);
            double* w1 = omega_q ? omega_q : ar.take<double>((size_t)nq * nm);
            double* w2 = omega_qp ? omega_qp : ar.take<double>((size_t)nqp * nm);
            double* w3 = omega_qpp ? omega_qpp : ar.take<double>((size_t)nq * nqp * nm);
            cd* E1 = ar.take<cd>((size_t)nq * nm * nm);
            cd* E2 = ar.take<cd>((size_t)nqp * nm * nm);
            cd* E3 = ar.take<cd>((size_t)nq * nqp * nm * nm);
            double* qpp = ar.take<double>((size_t)nq * nqp * 3);
            cd* phi3c = ar.take<cd>((size_t)n1 * n2 * m3);
            cd* P1 = ar.take<cd>((size_t)qb * n1);
            cd* P2 = ar.take<cd>((size_t)nqp * n2);
            cd* S = ar.take<cd>((size_t)qb * n2 * m3);
            cd* T = ar.take<cd>((size_t)qb * n2 * m3);
            cd* X = ar.take<cd>((size_t)nqp * m3);
            cd* Y = ar.take<cd>((size_t)nqp * m3);
            {
                Arena a1 = ar, a2 = ar, a3 = ar;
                phonon_dev(h, a1, &ph, rd, q_frac, nullptr, Mesh{1, 1, 1}, nq, omega_min, 0.0, w1, E1,
                           nullptr, nullptr, s);
                phonon_dev(h, a2, &ph, rd, qp_frac, nullptr, Mesh{1, 1, 1}, nqp, omega_min, 0.0, w2,
                           E2, nullptr, nullptr, s);
                if (ar.base) HIPCHK(h, launch_neg_pair_sum(q_frac, nq, qp_frac, nqp, qpp, s));
                phonon_dev(h, a3, &ph, rd, qpp, nullptr, Mesh{1, 1, 1}, nq * nqp, omega_min, 0.0, w3,
                           E3, nullptr, nullptr, s);
                ar.used = std::max(std::max(a1.used, a2.used), a3.used);
            }
            if (!ar.base) return;
            HIPCHK(h, launch_real_to_complex(sys->phi3, (int64_t)n1 * n2 * m3, phi3c, s));
            HIPCHK(h, launch_phase_table(qp_frac, nullptr, Mesh{1, 1, 1}, nqp, r2, n2, P2, n2, s));
            for (int64_t i0 = 0; i0 < nq; i0 += qb) {
                const int64_t nb = std::min(qb, nq - i0);
                HIPCHK(h, launch_phase_table(q_frac + 3 * i0, nullptr, Mesh{1, 1, 1}, nb, r1, n1, P1,
                                             n1, s));
                // S[i, (R', sa, s'b, s''c)] = sum_R e^{-i 2 pi q.R} Phi3[R, ...]
                Timer t1(h, s, "v3_stage1");
                HIPCHK(h, launch_zgemm(P1, n1, phi3c, (int64_t)n2 * m3, S, (int64_t)n2 * m3, nb,
                                       (int64_t)n2 * m3, n1, s));
                t1.done();
                HIPCHK(h, launch_v3_fold(S, nb, n2, nm, E1 + i0 * nm * nm, T, s));
                for (int64_t i = 0; i < nb; ++i) {
                    const int64_t iq = i0 + i;
                    // X[j, (nu, s'b, s''c)] = sum_R' e^{-i 2 pi q'.R'} T[i, R', ...]
                    Timer t2(h, s, "v3_stage2");
                    HIPCHK(h, launch_zgemm(P2, n2, T + i * n2 * m3, m3, X, m3, nqp, m3, n2, s));
                    t2.done();
                    HIPCHK(h, launch_v3_rot1(X, nqp, nm, E2, Y, s));
                    HIPCHK(h, launch_v3_rot2(Y, nqp, nm, E3 + iq * nqp * nm * nm,
                                             reinterpret_cast<cd*>(v3_out) + iq * nqp * m3, s));
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

phoebe_status phoebe_gpu_philox_uniform(void* handle, uint64_t seed, uint64_t offset, int64_t n,
                                        double* out, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        REQUIRE(h, n >= 0, "n < 0");
        if (n == 0) return;
        REQUIRE(h, out != nullptr, "out is NULL");
        HIPCHK(h, hipSetDevice(h->device));
        HIPCHK(h, launch_philox_uniform(seed, offset, n, out, s));
    });
}

phoebe_status phoebe_gpu_philox_randint(void* handle, uint64_t seed, uint64_t offset, int64_t n,
                                        int64_t hi, int32_t* out, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        REQUIRE(h, n >= 0, "n < 0");
        REQUIRE(h, hi >= 1 && hi <= 2147483647LL, "hi must be in [1, 2^31 - 1]");
        if (n == 0) return;
        REQUIRE(h, out != nullptr, "out is NULL");
        HIPCHK(h, hipSetDevice(h->device));
        HIPCHK(h, launch_philox_randint(seed, offset, n, hi, out, s));
    });
}

phoebe_status phoebe_gpu_mlp_init(void* handle, phoebe_precision prec, void* params, int32_t n_in,
                                  int32_t width, int32_t depth, uint64_t seed, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        REQUIRE(h, prec == PHOEBE_BF16 || prec == PHOEBE_FP64, "precision must be BF16 or FP64");
        REQUIRE(h, n_in >= 1 && width >= 1 && depth >= 0 && depth <= 16 && width <= 4096,
                "network shape out of range");
        REQUIRE(h, params != nullptr, "params is NULL");
        HIPCHK(h, hipSetDevice(h->device));
        const bool f64 = prec == PHOEBE_FP64;
        int64_t off = 0;
        int prev = n_in;
        for (int l = 0; l <= depth; ++l) {
            const int out = l == depth ? 1 : width;
            const int64_t nw = (int64_t)out * prev;
            HIPCHK(h, launch_uniform_fill(params, f64, seed, off, nw, std::sqrt((double)prev), s));
            char* b = static_cast<char*>(params) + (off + nw) * (f64 ? 8 : 4);
            HIPCHK(h, launch_zero(b, (size_t)out * (f64 ? 8 : 4), s));
            off += nw + out;
            prev = out;
        }
    });
}

phoebe_status phoebe_gpu_training_set(void* handle, const double* terms, const double* dweights,
                                      int64_t n_states, int64_t n_q, int32_t n_modes,
                                      double d_threshold, double c_frac, int64_t max_samples,
                                      uint64_t seed, int32_t* out_state, int32_t* out_q,
                                      int32_t* out_nu, float* out_y, int64_t cap, int64_t* n_out,
                                      double* c_out, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        REQUIRE(h, n_states >= 0 && n_q >= 1 && n_modes >= 1, "shape out of range");
        REQUIRE(h, std::isfinite(d_threshold) && d_threshold >= 0.0, "d_threshold must be >= 0");
        REQUIRE(h, std::isfinite(c_frac) && c_frac >= 0.0, "c_frac must be >= 0");
        REQUIRE(h, max_samples >= 1 && cap >= 0, "max_samples must be >= 1, cap >= 0");
        REQUIRE(h, n_out != nullptr, "n_out is NULL");
        *n_out = 0;
        if (c_out) *c_out = 0.0;
        if (n_states == 0) return;
        REQUIRE(h, terms && dweights, "terms/dweights is NULL");
        REQUIRE(h, cap == 0 || (out_state && out_q && out_nu && out_y), "outputs are NULL");
        const int64_t per = n_q * n_modes;
        const int64_t total = n_states * per;
        const int64_t nch = (total + kTsChunk - 1) / kTsChunk;
        REQUIRE(h, nch <= 2147483647LL && n_states <= 2147483647LL, "too many entries");
        HIPCHK(h, hipSetDevice(h->device));
        auto plan = [&](Arena& ar, double*& dmax, double*& partial, double*& stats, int32_t*& counts,
                        int64_t*& tot) {
            dmax = ar.take<double>(n_states);
            partial = ar.take<double>(2 * kTsBlocks);
            stats = ar.take<double>(2);
            counts = ar.take<int32_t>(nch);
            tot = ar.take<int64_t>(1);
        };
        double *dmax, *partial, *stats;
        int32_t* counts;
        int64_t* tot;
        Arena dry(nullptr);
        plan(dry, dmax, partial, stats, counts, tot);
        ensure_ws(h, dry.used);
        Arena ar(h->ws, h->ws_cap);
        plan(ar, dmax, partial, stats, counts, tot);
        HIPCHK(h, launch_ts_state_max(dweights, n_states, per, dmax, s));
        HIPCHK(h, launch_ts_stats(terms, dweights, dmax, n_states, per, d_threshold, partial, stats, s));
        double st[2] = {0.0, 0.0};
        HIPCHK(h, hipMemcpyAsync(st, stats, sizeof st, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        const double n_sel = st[0];
        if (n_sel == 0.0) return;
        const double c = c_frac * (st[1] / n_sel);
        const double p_keep = std::min(1.0, (double)max_samples / n_sel);
        if (c_out) *c_out = c;
        HIPCHK(h, launch_ts_count(dweights, dmax, n_states, per, d_threshold, seed, p_keep, counts, s));
        HIPCHK(h, launch_exclusive_scan(counts, nch, tot, s));
        HIPCHK(h, launch_ts_write(terms, dweights, dmax, n_states, per, n_modes, n_q, d_threshold,
                                  seed, p_keep, c, counts, cap, out_state, out_q, out_nu, out_y, s));
        int64_t kept = 0;
        HIPCHK(h, hipMemcpyAsync(&kept, tot, sizeof kept, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        *n_out = std::min(kept, cap);
    });
}

phoebe_status phoebe_gpu_gather_rows(void* handle, const void* src, int64_t n_src,
                                     int64_t row_bytes, const int32_t* idx, int64_t n, void* dst,
                                     void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        REQUIRE(h, n >= 0 && n_src >= 0, "negative count");
        REQUIRE(h, row_bytes >= 4 && row_bytes % 4 == 0, "row_bytes must be a positive multiple of 4");
        if (n == 0) return;
        REQUIRE(h, src && idx && dst, "src/idx/dst is NULL");
        REQUIRE(h, n_src >= 1, "n_src must be >= 1");
        HIPCHK(h, hipSetDevice(h->device));
        // indices are checked on the host before the gather runs
        std::vector<int32_t> ih(n);
        HIPCHK(h, hipMemcpyAsync(ih.data(), idx, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        for (int64_t i = 0; i < n; ++i)
            REQUIRE(h, ih[i] >= 0 && ih[i] < n_src, "idx[%lld] = %d out of range", (long long)i, ih[i]);
        HIPCHK(h, launch_gather_rows32(static_cast<const uint32_t*>(src), row_bytes / 4, idx, n,
                                       static_cast<uint32_t*>(dst), s));
    });
}

}  // extern "C"
