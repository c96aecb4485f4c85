// C ABI of the learned q-proposal: MLP forward/gradient/Adam, input features,
// and the proposal sampler that writes weighted per-k q lists for
// phoebe_gpu_scatter_rates.
#include "ext.hpp"
#include "host.hpp"
#include "mlp.hpp"

using namespace phx;

namespace {

struct Net {
    int n_in, width, depth;
    std::vector<std::pair<int, int>> shape;  // (out, in) per layer
    int64_t count = 0;
    Net(int ni, int w, int d) : n_in(ni), width(w), depth(d) {
        int prev = ni;
        for (int l = 0; l <= d; ++l) {
            const int out = l == d ? 1 : w;
            shape.push_back({out, prev});
            count += (int64_t)out * prev + out;
            prev = out;
        }
    }
};

void check_net(Handle* h, int n_in, int width, int depth) {
    REQUIRE(h, n_in >= 1 && width >= 1 && depth >= 0 && depth <= 16 && width <= 4096,
            "network shape out of range (n_in %d, width %d, depth %d)", n_in, width, depth);
}

template <class T>
void forward_impl(Handle* h, const Net& net, const T* P, const T* X, int64_t B, T* out,
                  std::vector<T*>& Z, std::vector<T*>& A, hipStream_t s) {
    const T* a = X;
    int64_t off = 0;
    for (size_t l = 0; l < net.shape.size(); ++l) {
        const int o = net.shape[l].first, i = net.shape[l].second;
        const T* W = P + off;
        const T* b = P + off + (int64_t)o * i;
        off += (int64_t)o * i + o;
        T* z = (l + 1 == net.shape.size() && out) ? out : Z[l];
        const bool hidden = l + 1 < net.shape.size();
        // hidden layers: z and silu(z) from the same pass
        HIPCHK(h, launch_mlp_gemm<T>(false, true, a, i, W, i, z, o, B, o, i, b, 0, s,
                                     hidden ? A[l] : nullptr));
        if (hidden) a = A[l];
    }
}

template <class T>
void grad_impl(Handle* h, const Net& net, const T* P, const T* X, const T* target, int64_t B,
               T* grad, double* loss, hipStream_t s) {
    const size_t L = net.shape.size();
    auto plan = [&](Arena& ar, std::vector<T*>& Z, std::vector<T*>& A, T*& dZ, T*& dA,
                    double*& sums) {
        for (size_t l = 0; l < L; ++l) {
            Z[l] = ar.take<T>((size_t)B * net.shape[l].first);
            A[l] = ar.take<T>((size_t)B * net.shape[l].first);
        }
        dZ = ar.take<T>((size_t)B * std::max(net.width, 1));
        dA = ar.take<T>((size_t)B * std::max(net.width, 1));
        sums = ar.take<double>(256);
    };
    std::vector<T*> Z(L), A(L);
    T *dZ, *dA;
    double* sums;
    Arena dry(nullptr);
    plan(dry, Z, A, dZ, dA, sums);
    ensure_ws(h, dry.used + 256);
    Arena ar(h->ws, h->ws_cap);
    plan(ar, Z, A, dZ, dA, sums);
    forward_impl<T>(h, net, P, X, B, nullptr, Z, A, s);
    const int nblk = (int)std::min<int64_t>(256, (B + 255) / 256);
    HIPCHK(h, launch_mse_grad<T>(Z[L - 1], target, dZ, B, sums, nblk, s));
    // offsets of each layer's parameters
    std::vector<int64_t> offs(L);
    int64_t off = 0;
    for (size_t l = 0; l < L; ++l) {
        offs[l] = off;
        off += (int64_t)net.shape[l].first * net.shape[l].second + net.shape[l].first;
    }
    for (int l = (int)L - 1; l >= 0; --l) {
        const int o = net.shape[l].first, i = net.shape[l].second;
        const T* aprev = l == 0 ? X : A[l - 1];
        // dW[o, i] = dZ^T[o, B] a_prev[B, i]
        HIPCHK(h, launch_mlp_gemm<T>(true, false, dZ, o, aprev, i, grad + offs[l], i, o, i, B, nullptr,
                                     0, s));
        HIPCHK(h, launch_colsum<T>(dZ, B, o, grad + offs[l] + (int64_t)o * i, s));
        if (l > 0) {
            // dA[B, i] = dZ[B, o] W[o, i]; dZ_prev = dA * silu'(z_prev)
            HIPCHK(h, launch_mlp_gemm<T>(false, false, dZ, o, P + offs[l], i, dA, i, B, i, o, nullptr,
                                         0, s));
            HIPCHK(h, launch_silu_bwd<T>(dA, Z[l - 1], dZ, B * i, s));
        }
    }
    if (loss) {
        std::vector<double> hs(nblk);
        HIPCHK(h, hipMemcpyAsync(hs.data(), sums, sizeof(double) * nblk, hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        double t = 0.0;
        for (double v : hs) t += v;
        *loss = t / (double)B;
    }
}

}  // namespace

extern "C" {

int64_t phoebe_gpu_mlp_param_count(int32_t n_in, int32_t width, int32_t depth) {
    if (n_in < 1 || width < 1 || depth < 0) return -1;
    return Net(n_in, width, depth).count;
}

phoebe_status phoebe_gpu_mlp_forward(void* handle, phoebe_precision prec, const void* params,
                                     int32_t n_in, int32_t width, int32_t depth, const void* X,
                                     int64_t batch, void* out, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        check_net(h, n_in, width, depth);
        REQUIRE(h, prec == PHOEBE_FP64 || prec == PHOEBE_BF16, "MLP precision must be FP64 or BF16");
        REQUIRE(h, batch >= 0, "batch < 0");
        if (batch == 0) return;
        REQUIRE(h, params && X && out, "params/X/out is NULL");
        HIPCHK(h, hipSetDevice(h->device));
        const Net net(n_in, width, depth);
        auto go = [&](auto* tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            std::vector<T*> Z(net.shape.size()), A(net.shape.size());
            auto plan = [&](Arena& ar) {
                for (size_t l = 0; l < net.shape.size(); ++l) {
                    Z[l] = ar.take<T>((size_t)batch * net.shape[l].first);
                    A[l] = ar.take<T>((size_t)batch * net.shape[l].first);
                }
            };
            Arena dry(nullptr);
            plan(dry);
            ensure_ws(h, dry.used + 256);
            Arena ar(h->ws, h->ws_cap);
            plan(ar);
            forward_impl<T>(h, net, (const T*)params, (const T*)X, batch, (T*)out, Z, A, s);
        };
        if (prec == PHOEBE_FP64)
            go((double*)nullptr);
        else
            go((float*)nullptr);
        HIPCHK(h, hipGetLastError());
    });
}

phoebe_status phoebe_gpu_mlp_grad(void* handle, phoebe_precision prec, const void* params,
                                  int32_t n_in, int32_t width, int32_t depth, const void* X,
                                  const void* target, int64_t batch, void* grad, double* loss,
                                  void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        check_net(h, n_in, width, depth);
        REQUIRE(h, prec == PHOEBE_FP64 || prec == PHOEBE_BF16, "MLP precision must be FP64 or BF16");
        REQUIRE(h, batch >= 1, "batch < 1");
        REQUIRE(h, params && X && target && grad, "params/X/target/grad is NULL");
        HIPCHK(h, hipSetDevice(h->device));
        const Net net(n_in, width, depth);
        if (prec == PHOEBE_FP64)
            grad_impl<double>(h, net, (const double*)params, (const double*)X, (const double*)target,
                              batch, (double*)grad, loss, s);
        else
            grad_impl<float>(h, net, (const float*)params, (const float*)X, (const float*)target,
                             batch, (float*)grad, loss, s);
        HIPCHK(h, hipGetLastError());
    });
}

phoebe_status phoebe_gpu_mlp_adam(void* handle, float* params, const float* grad, float* m,
                                  float* v, int64_t n, int32_t step, double lr, double beta1,
                                  double beta2, double eps, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        REQUIRE(h, params && grad && m && v && n >= 0 && step >= 1, "bad Adam arguments");
        REQUIRE(h, beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps >= 0 && lr >= 0,
                "Adam hyper-parameters out of range");
        HIPCHK(h, hipSetDevice(h->device));
        if (n > 0) HIPCHK(h, launch_adam(params, grad, m, v, n, step, lr, beta1, beta2, eps, s));
    });
}

int32_t phoebe_gpu_mlp_feature_count(int32_t n_modes, int32_t n_harm) {
    if (n_modes < 1 || n_harm < 0 || n_harm > 16) return -1;
    return feature_count(n_modes, n_harm);
}

phoebe_status phoebe_gpu_mlp_features(void* handle, phoebe_precision prec, const int32_t mesh[3],
                                      int32_t n_modes, int32_t n_harm, const int32_t* k_idx,
                                      const double* eps, const int32_t* q_idx, const int32_t* nu,
                                      int64_t batch, double e0, double escale, void* X,
                                      void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        REQUIRE(h, mesh && mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "bad mesh");
        REQUIRE(h, n_modes >= 1 && escale > 0.0, "n_modes >= 1 and escale > 0 required");
        REQUIRE(h, n_harm >= 0 && n_harm <= 16, "n_harm must be in [0, 16]");
        REQUIRE(h, prec == PHOEBE_FP64 || prec == PHOEBE_BF16, "precision must be FP64 or BF16");
        if (batch == 0) return;
        REQUIRE(h, batch > 0 && k_idx && eps && q_idx && nu && X, "NULL arrays");
        HIPCHK(h, hipSetDevice(h->device));
        const Mesh m{mesh[0], mesh[1], mesh[2]};
        if (prec == PHOEBE_FP64)
            HIPCHK(h, launch_features<double>(k_idx, eps, q_idx, nu, batch, m, n_modes, n_harm, e0,
                                              escale, (double*)X, s));
        else
            HIPCHK(h, launch_features<float>(k_idx, eps, q_idx, nu, batch, m, n_modes, n_harm, e0,
                                             escale, (float*)X, s));
    });
}

phoebe_status phoebe_gpu_propose_q(void* handle, const int32_t mesh[3], int32_t n_modes,
                                   int32_t n_harm, const int32_t* k_idx, const double* eps_k, int64_t nk,
                                   const double* dweights, const float* params, int32_t width,
                                   int32_t depth, double e0, double escale, double d_threshold,
                                   double mix, int32_t S, const double* uniforms, int64_t* q_off,
                                   int32_t* q_idx, double* q_w, void* stream) {
    if (!handle) return PHOEBE_E_INVALID;
    Handle* h = static_cast<Handle*>(handle);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return run(h, __func__, [&] {
        REQUIRE(h, mesh && mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1, "bad mesh");
        REQUIRE(h, n_modes >= 1 && escale > 0.0 && S >= 1, "n_modes >= 1, escale > 0, S >= 1");
        REQUIRE(h, mix > 0.0 && mix <= 1.0, "mix must be in (0, 1]: the uniform share keeps the "
                                            "proposal's support full");
        REQUIRE(h, d_threshold >= 0.0 && d_threshold < 1.0, "d_threshold must be in [0, 1)");
        REQUIRE(h, n_harm >= 0 && n_harm <= 16, "n_harm must be in [0, 16]");
        if (nk == 0) return;
        REQUIRE(h, nk > 0 && k_idx && eps_k && dweights && uniforms && q_off && q_idx && q_w,
                "NULL arrays");
        const int n_in = feature_count(n_modes, n_harm);
        if (params) check_net(h, n_in, width, depth);
        HIPCHK(h, hipSetDevice(h->device));
        const Mesh m{mesh[0], mesh[1], mesh[2]};
        const int64_t N = (int64_t)m.n0 * m.n1 * m.n2;
        const int64_t NR = N * n_modes;
        REQUIRE(h, NR < ((int64_t)1 << 31), "mesh x modes too large");
        for (int64_t i = 0; i < nk; ++i)
            REQUIRE(h, k_idx[i] >= 0 && k_idx[i] < N, "k_idx[%lld] not a mesh index", (long long)i);
        REQUIRE(h, nk * NR < ((int64_t)1 << 31), "k count x mesh x modes too large for one call");
        // every k at once: the selection over all rows, the network in batches of at most
        // `chunk` listed entries, then one sampler work-group per k
        const int64_t chunk = 262144;
        const Net net(n_in, params ? width : 1, params ? depth : 0);
        std::vector<float*> Z(net.shape.size()), A(net.shape.size());
        float *X = nullptr, *y = nullptr;
        double *p = nullptr, *E = nullptr, *dmax = nullptr, *ek = nullptr;
        int32_t *list = nullptr, *counts = nullptr, *kd = nullptr;
        int64_t* total = nullptr;
        const int64_t nch = select_rows_chunks(nk, NR);
        auto plan = [&](Arena& ar) {
            p = ar.take<double>((size_t)nk * N);
            kd = ar.take<int32_t>((size_t)nk);
            ek = ar.take<double>((size_t)nk);
            if (params) {
                E = ar.take<double>((size_t)nk * NR);
                dmax = ar.take<double>((size_t)nk);
                counts = ar.take<int32_t>((size_t)nch);
                total = ar.take<int64_t>(1);
                list = ar.take<int32_t>((size_t)nk * NR);
                X = ar.take<float>((size_t)chunk * n_in);
                for (size_t l = 0; l < net.shape.size(); ++l) {
                    Z[l] = ar.take<float>((size_t)chunk * net.shape[l].first);
                    A[l] = ar.take<float>((size_t)chunk * net.shape[l].first);
                }
                y = ar.take<float>((size_t)chunk);
            }
        };
        Arena dry(nullptr);
        plan(dry);
        ensure_ws(h, dry.used + 256);
        Arena ar(h->ws, h->ws_cap);
        plan(ar);
        std::vector<int64_t> offs(nk + 1);
        for (int64_t i = 0; i <= nk; ++i) offs[i] = i * S;
        HIPCHK(h, hipMemcpyAsync(q_off, offs.data(), sizeof(int64_t) * (nk + 1), hipMemcpyHostToDevice, s));
        Timer t(h, s, "mlp_proposal");
        if (!params) {
            HIPCHK(h, launch_sum_modes(dweights, nk * N, n_modes, p, s));
        } else {
            HIPCHK(h, hipMemcpyAsync(kd, k_idx, sizeof(int32_t) * nk, hipMemcpyHostToDevice, s));
            HIPCHK(h, hipMemcpyAsync(ek, eps_k, sizeof(double) * nk, hipMemcpyHostToDevice, s));
            // evaluate the network only where the smearing weight matters
            HIPCHK(h, launch_ts_state_max(dweights, nk, NR, dmax, s));
            HIPCHK(h, launch_select_rows(dweights, dmax, nk, NR, d_threshold, counts, total, list, s));
            HIPCHK(h, launch_zero(E, (size_t)nk * NR * sizeof(double), s));
            int64_t cnt = 0;
            HIPCHK(h, hipMemcpyAsync(&cnt, total, sizeof cnt, hipMemcpyDeviceToHost, s));
            HIPCHK(h, hipStreamSynchronize(s));
            for (int64_t c0 = 0; c0 < cnt; c0 += chunk) {
                const int64_t nc = std::min<int64_t>(chunk, cnt - c0);
                HIPCHK(h, launch_features_flat(kd, ek, list + c0, nc, NR, m, n_modes, n_harm, e0,
                                               escale, X, s));
                forward_impl<float>(h, net, params, X, nc, y, Z, A, s);
                HIPCHK(h, launch_weight_list(dweights, list + c0, y, nc, E, s));
            }
            HIPCHK(h, launch_sum_modes(E, nk * N, n_modes, p, s));
        }
        HIPCHK(h, launch_sample(p, N, mix, uniforms, S, q_idx, q_w, nk, s));
        t.done();
        HIPCHK(h, hipStreamSynchronize(s));  // host offsets are read before return
        flush_timing(h, s);
    });
}

}  // extern "C"
