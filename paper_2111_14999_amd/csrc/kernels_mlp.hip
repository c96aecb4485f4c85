// Learned q-proposal: multilayer perceptron training and inference kernels,
// the proposal/inverse-CDF sampler and the importance-sampling weights.
//
// Network: z_l = W_l a_{l-1} + b_l, a_l = silu(z_l) for hidden layers, linear
// output; parameters packed per layer as W_l [out, in] then b_l [out].
// Two arithmetic paths: BF16 operands on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation (float storage), and an FP64 path on v_mfma_f64_16x16x4f64
// (double storage) used to check gradients against the FP64 oracle.
#include <algorithm>

#include "ext.hpp"
#include "mlp.hpp"

namespace phx {

static inline int gridm(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535 * 16) g = 65535 * 16;
    if (g < 1) g = 1;
    return (int)g;
}

__device__ inline uint16_t f2bf(float x) {
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + (((u >> 16) & 1u) + 0x7FFFu)) >> 16);
}

typedef short s8m __attribute__((ext_vector_type(8)));
typedef __bf16 bf8m __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// C[M, N] = op(A)[M, K] op(B)[K, N] (+ bias[N]) (+ C if accumulate)
//   A(i, k) = TA ? A[k lda + i] : A[i lda + k];  B(k, j) = TB ? B[j ldb + k] : B[k ldb + j]
// Work-group: 4 waves side by side along N, each 2 x 2 tiles of 16 x 16.
// ---------------------------------------------------------------------------
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void mlp_gemm_bf16(const float* __restrict__ A, int64_t lda,
                                                     const float* __restrict__ B, int64_t ldb,
                                                     float* __restrict__ C, int64_t ldc, int64_t M,
                                                     int64_t N, int64_t K,
                                                     const float* __restrict__ bias, int accumulate) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * 32;
    const int64_t n0 = ((int64_t)blockIdx.x * 4 + wave) * 32;
    if (n0 >= N) return;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[i][t] = f4{0, 0, 0, 0};
    for (int64_t k0 = 0; k0 < K; k0 += 32) {
        s8m a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int64_t row = m0 + 16 * i + li;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t k = k0 + 8 * lk + j;
                float v = 0.f;
                if (row < M && k < K) v = TA ? A[k * lda + row] : A[row * lda + k];
                a[i][j] = (short)f2bf(v);
            }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int64_t col = n0 + 16 * t + li;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t k = k0 + 8 * lk + j;
                float v = 0.f;
                if (col < N && k < K) v = TB ? B[col * ldb + k] : B[k * ldb + col];
                b[t][j] = (short)f2bf(v);
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf8m, a[i]), __builtin_bit_cast(bf8m, b[t]), acc[i][t], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + 16 * i + 4 * lk + v;
                const int64_t col = n0 + 16 * t + li;
                if (row < M && col < N) {
                    float r = acc[i][t][v];
                    if (bias) r += bias[col];
                    if (accumulate) r += C[row * ldc + col];
                    C[row * ldc + col] = r;
                }
            }
}

// The same BF16 product, LDS-tiled: a work-group of 4 waves owns a 128 x 128 tile
// of C (each wave 64 x 64: 4 x 4 MFMA tiles); per 32-wide K step the A and B tiles
// are converted to BF16 once, staged in LDS (rows padded to 40 BF16 so the 16-byte
// fragment reads of a 16-lane group hit distinct banks) and read from there by
// every wave.  The K steps, the MFMA and the epilogue are those of mlp_gemm_bf16,
// so the results are the same bits.  With act set, silu(C) is written there too.
constexpr int kGT = 128;   // tile rows and columns
constexpr int kGK = 32;    // K step
constexpr int kGLd = 40;   // LDS row stride (BF16 elements)

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void mlp_gemm_bf16_tiled(
    const float* __restrict__ A, int64_t lda, const float* __restrict__ B, int64_t ldb,
    float* __restrict__ C, int64_t ldc, int64_t M, int64_t N, int64_t K,
    const float* __restrict__ bias, int accumulate, float* __restrict__ act) {
    __shared__ __align__(16) uint16_t sA[kGT * kGLd];
    __shared__ __align__(16) uint16_t sB[kGT * kGLd];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.y * kGT, n0 = (int64_t)blockIdx.x * kGT;
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[i][t] = f4{0, 0, 0, 0};
    // element (row r of the tile, k) of op(A) and (k, column c) of op(B)
    auto a_at = [&](int64_t row, int64_t k) -> float {
        return (row < M && k < K) ? (TA ? A[k * lda + row] : A[row * lda + k]) : 0.f;
    };
    auto b_at = [&](int64_t col, int64_t k) -> float {
        return (col < N && k < K) ? (TB ? B[col * ldb + k] : B[k * ldb + col]) : 0.f;
    };
    for (int64_t k0 = 0; k0 < K; k0 += kGK) {
        // stage: each thread converts 8 (row, k pair) entries of each tile; pairs
        // along k for row-major operands, along the rows for transposed ones, so
        // that neighbouring threads read neighbouring addresses
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = tid + 256 * j;
            const int r = TA ? (e & (kGT - 1)) : (e >> 4);
            const int kp = TA ? (e >> 7) : (e & 15);
            const int64_t row = m0 + r, k = k0 + 2 * kp;
            const uint32_t v = (uint32_t)f2bf(a_at(row, k)) | ((uint32_t)f2bf(a_at(row, k + 1)) << 16);
            *reinterpret_cast<uint32_t*>(&sA[r * kGLd + 2 * kp]) = v;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = tid + 256 * j;
            const int c = TB ? (e >> 4) : (e & (kGT - 1));
            const int kp = TB ? (e & 15) : (e >> 7);
            const int64_t col = n0 + c, k = k0 + 2 * kp;
            const uint32_t v = (uint32_t)f2bf(b_at(col, k)) | ((uint32_t)f2bf(b_at(col, k + 1)) << 16);
            *reinterpret_cast<uint32_t*>(&sB[c * kGLd + 2 * kp]) = v;
        }
        __syncthreads();
        s8m a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a[i] = *reinterpret_cast<const s8m*>(&sA[(64 * wm + 16 * i + li) * kGLd + 8 * lk]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            b[t] = *reinterpret_cast<const s8m*>(&sB[(64 * wn + 16 * t + li) * kGLd + 8 * lk]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf8m, a[i]), __builtin_bit_cast(bf8m, b[t]), acc[i][t], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + 64 * wm + 16 * i + 4 * lk + v;
                const int64_t col = n0 + 64 * wn + 16 * t + li;
                if (row < M && col < N) {
                    float r = acc[i][t][v];
                    if (bias) r += bias[col];
                    if (accumulate) r += C[row * ldc + col];
                    C[row * ldc + col] = r;
                    if (act) act[row * ldc + col] = r / (1.0f + exp(-r));
                }
            }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void mlp_gemm_f64(const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb,
                                                    double* __restrict__ C, int64_t ldc, int64_t M,
                                                    int64_t N, int64_t K,
                                                    const double* __restrict__ bias, int accumulate) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * 32;
    const int64_t n0 = ((int64_t)blockIdx.x * 4 + wave) * 32;
    if (n0 >= N) return;
    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[i][t] = d4{0, 0, 0, 0};
    for (int64_t k0 = 0; k0 < K; k0 += 4) {
        const int64_t k = k0 + lk;
        double a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int64_t row = m0 + 16 * i + li;
            a[i] = (row < M && k < K) ? (TA ? A[k * lda + row] : A[row * lda + k]) : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int64_t col = n0 + 16 * t + li;
            b[t] = (col < N && k < K) ? (TB ? B[col * ldb + k] : B[k * ldb + col]) : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int t = 0; t < 2; ++t)
                acc[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[t], acc[i][t], 0, 0, 0);
    }
    // f64 MFMA result v of lane group lk is row lk + 4v
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + 16 * i + lk + 4 * v;
                const int64_t col = n0 + 16 * t + li;
                if (row < M && col < N) {
                    double r = acc[i][t][v];
                    if (bias) r += bias[col];
                    if (accumulate) r += C[row * ldc + col];
                    C[row * ldc + col] = r;
                }
            }
}

template <class T>
hipError_t launch_mlp_gemm(bool ta, bool tb, const T* A, int64_t lda, const T* B, int64_t ldb, T* C,
                           int64_t ldc, int64_t M, int64_t N, int64_t K, const T* bias, int acc,
                           hipStream_t s, T* act) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if constexpr (sizeof(T) == 4) {
        // large products (the network over many samples) on the tiled kernel, where its
        // 128 x 128 tiles still make enough work-groups to fill the chip
        if (N >= 64 && ((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT) >= 512) {
            dim3 g((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT));
            if (g.y > 65535) return hipErrorInvalidValue;
#define PHX_GT(TAv, TBv)                                                                         \
            if (ta == TAv && tb == TBv) {                                                        \
                hipLaunchKernelGGL((mlp_gemm_bf16_tiled<TAv, TBv>), g, dim3(256), 0, s,          \
                                   (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc,   \
                                   M, N, K, (const float*)bias, acc, (float*)act);               \
                return hipGetLastError();                                                        \
            }
            PHX_GT(false, false) PHX_GT(false, true) PHX_GT(true, false) PHX_GT(true, true)
#undef PHX_GT
        }
    }
    if (act) {  // the small products: the activation as its own pass
        hipError_t e = launch_mlp_gemm<T>(ta, tb, A, lda, B, ldb, C, ldc, M, N, K, bias, acc, s);
        if (e != hipSuccess) return e;
        if (ldc != N) return hipErrorInvalidValue;
        return launch_silu_fwd<T>(C, act, M * N, s);
    }
    dim3 grid((unsigned)((N + 127) / 128), (unsigned)((M + 31) / 32));
    if (grid.y > 65535) return hipErrorInvalidValue;
#define PHX_GO(TAv, TBv)                                                                        \
    if (ta == TAv && tb == TBv) {                                                               \
        if constexpr (sizeof(T) == 4)                                                           \
            hipLaunchKernelGGL((mlp_gemm_bf16<TAv, TBv>), grid, dim3(256), 0, s,                  \
                               (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc, M, N, \
                               K, (const float*)bias, acc);                                      \
        else                                                                                    \
            hipLaunchKernelGGL((mlp_gemm_f64<TAv, TBv>), grid, dim3(256), 0, s,                   \
                               (const double*)A, lda, (const double*)B, ldb, (double*)C, ldc, M, \
                               N, K, (const double*)bias, acc);                                  \
        return hipGetLastError();                                                               \
    }
    PHX_GO(false, false) PHX_GO(false, true) PHX_GO(true, false) PHX_GO(true, true)
#undef PHX_GO
    return hipErrorInvalidValue;
}
template hipError_t launch_mlp_gemm<float>(bool, bool, const float*, int64_t, const float*, int64_t,
                                           float*, int64_t, int64_t, int64_t, int64_t, const float*,
                                           int, hipStream_t, float*);
template hipError_t launch_mlp_gemm<double>(bool, bool, const double*, int64_t, const double*,
                                            int64_t, double*, int64_t, int64_t, int64_t, int64_t,
                                            const double*, int, hipStream_t, double*);

// ---------------------------------------------------------------------------
// elementwise pieces
// ---------------------------------------------------------------------------
template <class T>
__global__ void silu_fwd_kernel(const T* z, T* a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T x = z[i];
        a[i] = x / ((T)1 + exp(-x));
    }
}
template <class T>
__global__ void silu_bwd_kernel(const T* da, const T* z, T* dz, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T x = z[i];
        const T sg = (T)1 / ((T)1 + exp(-x));
        dz[i] = da[i] * sg * ((T)1 + x * ((T)1 - sg));
    }
}
// dY = 2 (Y - t) / B; squared errors summed per block into sums[block]
template <class T>
__global__ void mse_grad_kernel(const T* y, const T* t, T* dy, int64_t B, double* sums) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < B;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T r = y[i] - t[i];
        dy[i] = (T)2 * r / (T)B;
        acc += (double)r * (double)r;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = sh[0];
}
// db[j] = sum_b dZ[b, j]
template <class T>
__global__ __launch_bounds__(256) void colsum_kernel(const T* dz, int64_t B, int64_t N, T* db) {
    __shared__ double sh[256];
    const int64_t j = blockIdx.x;
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < B; b += 256) acc += (double)dz[b * N + j];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[j] = (T)sh[0];
}

template <class T>
hipError_t launch_silu_fwd(const T* z, T* a, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(silu_fwd_kernel<T>, dim3(gridm(n, 256)), dim3(256), 0, s, z, a, n);
    return hipGetLastError();
}
template <class T>
hipError_t launch_silu_bwd(const T* da, const T* z, T* dz, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(silu_bwd_kernel<T>, dim3(gridm(n, 256)), dim3(256), 0, s, da, z, dz, n);
    return hipGetLastError();
}
template <class T>
hipError_t launch_mse_grad(const T* y, const T* t, T* dy, int64_t B, double* sums, int nblk,
                           hipStream_t s) {
    hipLaunchKernelGGL(mse_grad_kernel<T>, dim3(nblk), dim3(256), 0, s, y, t, dy, B, sums);
    return hipGetLastError();
}
template <class T>
hipError_t launch_colsum(const T* dz, int64_t B, int64_t N, T* db, hipStream_t s) {
    hipLaunchKernelGGL(colsum_kernel<T>, dim3((unsigned)N), dim3(256), 0, s, dz, B, N, db);
    return hipGetLastError();
}
#define PHX_INST(T)                                                                              \
    template hipError_t launch_silu_fwd<T>(const T*, T*, int64_t, hipStream_t);                  \
    template hipError_t launch_silu_bwd<T>(const T*, const T*, T*, int64_t, hipStream_t);         \
    template hipError_t launch_mse_grad<T>(const T*, const T*, T*, int64_t, double*, int,          \
                                           hipStream_t);                                          \
    template hipError_t launch_colsum<T>(const T*, int64_t, int64_t, T*, hipStream_t);
PHX_INST(float)
PHX_INST(double)
#undef PHX_INST

// Adam on FP32 master parameters (Kingma & Ba, bias-corrected moments)
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, double lr,
                            double b1, double b2, double eps, double c1, double c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double gi = g[i];
        const double mi = b1 * m[i] + (1.0 - b1) * gi;
        const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
        m[i] = (float)mi;
        v[i] = (float)vi;
        p[i] = (float)(p[i] - lr * (mi / c1) / (sqrt(vi / c2) + eps));
    }
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int t, double lr,
                       double b1, double b2, double eps, hipStream_t s) {
    const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    hipLaunchKernelGGL(adam_kernel, dim3(gridm(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Network inputs of one sample (k, band energy, q, mode nu):
//   n_harm = 0: [k (3 crystal coords), (eps - e0)/escale, q (3), one-hot(nu)]
//   n_harm > 0: [(eps - e0)/escale, one-hot(nu), then for h = 1..n_harm
//                cos, sin of 2 pi h k_d (3 + 3) and of 2 pi h q_d (3 + 3)]
// The periodic form gives the network the Fourier harmonics in which the
// Wannier-gauge coupling is band-limited; h i_d mod N_d is reduced exactly.
// ---------------------------------------------------------------------------
__host__ __device__ inline int n_features(int nm, int n_harm) {
    return n_harm == 0 ? 7 + nm : 1 + nm + 12 * n_harm;
}

template <class T>
__device__ inline void write_features(T* x, int k0, int k1, int k2, int q0, int q1, int q2, int nu,
                                      double e, Mesh mesh, int nm, int n_harm) {
    if (n_harm == 0) {
        x[0] = (T)((double)k0 / mesh.n0);
        x[1] = (T)((double)k1 / mesh.n1);
        x[2] = (T)((double)k2 / mesh.n2);
        x[3] = (T)e;
        x[4] = (T)((double)q0 / mesh.n0);
        x[5] = (T)((double)q1 / mesh.n1);
        x[6] = (T)((double)q2 / mesh.n2);
        for (int v = 0; v < nm; ++v) x[7 + v] = (T)(v == nu ? 1 : 0);
        return;
    }
    x[0] = (T)e;
    for (int v = 0; v < nm; ++v) x[1 + v] = (T)(v == nu ? 1 : 0);
    const int idx[6] = {k0, k1, k2, q0, q1, q2};
    const int Ns[6] = {mesh.n0, mesh.n1, mesh.n2, mesh.n0, mesh.n1, mesh.n2};
    T* y = x + 1 + nm;
    for (int h = 1; h <= n_harm; ++h)
        for (int d = 0; d < 6; ++d) {
            const int a = (int)(((int64_t)h * idx[d]) % Ns[d]);
            double sn, cs;
            sincospi(2.0 * (double)a / Ns[d], &sn, &cs);
            y[0] = (T)cs;
            y[1] = (T)sn;
            y += 2;
        }
}

template <class T>
__global__ void features_kernel(const int32_t* k_idx, const double* eps, const int32_t* q_idx,
                                const int32_t* nu, int64_t B, Mesh mesh, int nm, int n_harm,
                                double e0, double escale, T* X) {
    const int nin = n_features(nm, n_harm);
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < B;
         b += (int64_t)gridDim.x * blockDim.x) {
        int k0, k1, k2, q0, q1, q2;
        mesh_triple(k_idx[b], mesh, k0, k1, k2);
        mesh_triple(q_idx[b], mesh, q0, q1, q2);
        write_features<T>(X + b * nin, k0, k1, k2, q0, q1, q2, nu[b], (eps[b] - e0) / escale, mesh,
                          nm, n_harm);
    }
}

template <class T>
hipError_t launch_features(const int32_t* k_idx, const double* eps, const int32_t* q_idx,
                           const int32_t* nu, int64_t B, Mesh mesh, int nm, int n_harm, double e0,
                           double escale, T* X, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel<T>, dim3(gridm(B, 256)), dim3(256), 0, s, k_idx, eps, q_idx,
                       nu, B, mesh, nm, n_harm, e0, escale, X);
    return hipGetLastError();
}
template hipError_t launch_features<float>(const int32_t*, const double*, const int32_t*,
                                           const int32_t*, int64_t, Mesh, int, int, double, double,
                                           float*, hipStream_t);
template hipError_t launch_features<double>(const int32_t*, const double*, const int32_t*,
                                            const int32_t*, int64_t, Mesh, int, int, double, double,
                                            double*, hipStream_t);

int feature_count(int nm, int n_harm) { return n_features(nm, n_harm); }

// p_raw[q] = sum_nu max(exp(y[q nm + nu]) - c, 0)
__global__ void proposal_raw_kernel(const float* y, int64_t nq, int nm, double c, double* p) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nq;
         q += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int v = 0; v < nm; ++v) {
            const double e = exp(fmin((double)y[q * nm + v], 80.0)) - c;
            acc += e > 0.0 ? e : 0.0;
        }
        p[q] = acc;
    }
}

hipError_t launch_proposal_raw(const float* y, int64_t nq, int nm, double c, double* p,
                               hipStream_t s) {
    hipLaunchKernelGGL(proposal_raw_kernel, dim3(gridm(nq, 256)), dim3(256), 0, s, y, nq, nm, c, p);
    return hipGetLastError();
}

// E[list[i]] = D[list[i]] exp(y[i])
__global__ void weight_list_kernel(const double* D, const int32_t* list, const float* y, int64_t n,
                                   double* E) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = list[i];
        E[r] = D[r] * exp(fmin((double)y[i], 80.0));
    }
}

// p_raw[q] = sum_nu E[q nm + nu] (fixed order)
__global__ void sum_modes_kernel(const double* E, int64_t N, int nm, double* p) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < N;
         q += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int v = 0; v < nm; ++v) acc += E[q * nm + v];
        p[q] = acc;
    }
}

hipError_t launch_weight_list(const double* D, const int32_t* list, const float* y, int64_t n,
                              double* E, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(weight_list_kernel, dim3(gridm(n, 256)), dim3(256), 0, s, D, list, y, n, E);
    return hipGetLastError();
}
hipError_t launch_sum_modes(const double* E, int64_t N, int nm, double* p, hipStream_t s) {
    hipLaunchKernelGGL(sum_modes_kernel, dim3(gridm(N, 256)), dim3(256), 0, s, E, N, nm, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The proposal for many k at once: entries f = k NR + (q nm + nu) of D [nk, NR]
// with D > thr x max over the k's row are listed in flat order (per-chunk
// counts, an exclusive scan, then the writes), so the network runs over the
// listed entries of every k in a few large batches.
// ---------------------------------------------------------------------------
constexpr int kSelChunk = 4096;

__global__ __launch_bounds__(256) void sel_count_kernel(const double* D, const double* dmax,
                                                        int64_t total, int64_t NR, double thr,
                                                        int32_t* counts) {
    __shared__ int sm[4];
    const int64_t c0 = (int64_t)blockIdx.x * kSelChunk;
    int n = 0;
    for (int i = threadIdx.x; i < kSelChunk; i += 256) {
        const int64_t f = c0 + i;
        if (f < total && D[f] > thr * dmax[f / NR]) ++n;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

__global__ __launch_bounds__(256) void sel_write_kernel(const double* D, const double* dmax,
                                                        int64_t total, int64_t NR, double thr,
                                                        const int32_t* offsets, int32_t* list) {
    __shared__ int wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kSelChunk;
    int64_t base = offsets[blockIdx.x];
    for (int i0 = 0; i0 < kSelChunk; i0 += 256) {
        const int64_t f = c0 + i0 + tid;
        const bool keep = f < total && D[f] > thr * dmax[f / NR];
        const uint64_t bal = __ballot(keep);
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (keep) list[base + before + __popcll(bal & ((1ull << lane) - 1ull))] = (int32_t)f;
        base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

hipError_t launch_select_rows(const double* D, const double* dmax, int64_t nk, int64_t NR,
                              double thr, int32_t* counts, int64_t* total_out, int32_t* list,
                              hipStream_t s) {
    const int64_t total = nk * NR;
    const int64_t nch = (total + kSelChunk - 1) / kSelChunk;
    if (nch <= 0) return hipSuccess;
    if (nch > 2147483647LL || total > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sel_count_kernel, dim3((unsigned)nch), dim3(256), 0, s, D, dmax, total, NR,
                       thr, counts);
    hipError_t e = launch_exclusive_scan(counts, nch, total_out, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sel_write_kernel, dim3((unsigned)nch), dim3(256), 0, s, D, dmax, total, NR,
                       thr, counts, list);
    return hipGetLastError();
}
int64_t select_rows_chunks(int64_t nk, int64_t NR) { return (nk * NR + kSelChunk - 1) / kSelChunk; }

// features of listed flat entries f = k NR + q nm + nu; k's mesh index and band
// energy from per-k device arrays
__global__ void features_flat_kernel(const int32_t* kmesh, const double* epsk, const int32_t* list,
                                     int64_t n, int64_t NR, Mesh mesh, int nm, int n_harm,
                                     double e0, double escale, float* X) {
    const int nin = n_features(nm, n_harm);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = list[i];
        const int64_t kl = f / NR, r = f - kl * NR;
        const int64_t q = r / nm;
        const int nu = (int)(r - q * nm);
        int k0, k1, k2, a0, a1, a2;
        mesh_triple(kmesh[kl], mesh, k0, k1, k2);
        mesh_triple(q, mesh, a0, a1, a2);
        write_features<float>(X + i * nin, k0, k1, k2, a0, a1, a2, nu, (epsk[kl] - e0) / escale,
                              mesh, nm, n_harm);
    }
}

hipError_t launch_features_flat(const int32_t* kmesh, const double* epsk, const int32_t* list,
                                int64_t n, int64_t NR, Mesh mesh, int nm, int n_harm, double e0,
                                double escale, float* X, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_flat_kernel, dim3(gridm(n, 256)), dim3(256), 0, s, kmesh, epsk,
                       list, n, NR, mesh, nm, n_harm, e0, escale, X);
    return hipGetLastError();
}

// One work-group per k: normalise p_raw (mixed with the uniform distribution),
// build the CDF by an ordered FP64 scan, draw S points by inverse CDF of the
// given uniforms and write the importance weights 1 / (N S p(q)).
__global__ __launch_bounds__(1024) void sample_kernel(double* p, int64_t N, double mix,
                                                      const double* u, int S, int32_t* q_idx,
                                                      double* q_w) {
    // work-group j samples for the j-th k: its row of p and its S uniforms and outputs
    p += (int64_t)blockIdx.x * N;
    u += (int64_t)blockIdx.x * S;
    q_idx += (int64_t)blockIdx.x * S;
    q_w += (int64_t)blockIdx.x * S;
    __shared__ double wsum[16];
    __shared__ double base_sh;
    __shared__ double total_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // total of p_raw
    double loc = 0.0;
    for (int64_t i = tid; i < N; i += 1024) loc += p[i];
    for (int o = 32; o > 0; o >>= 1) loc += __shfl_xor(loc, o, 64);
    if (lane == 0) wsum[wave] = loc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += wsum[w];
        total_sh = t;
        base_sh = 0.0;
    }
    __syncthreads();
    const double tot = total_sh;
    const double a = tot > 0.0 ? (1.0 - mix) / tot : 0.0;
    const double b = tot > 0.0 ? mix / (double)N : 1.0 / (double)N;
    // p <- normalised mixture; then in-place inclusive scan (CDF)
    for (int64_t c0 = 0; c0 < N; c0 += 1024) {
        const int64_t i = c0 + tid;
        double v = i < N ? a * p[i] + b : 0.0;
        double x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        __syncthreads();
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        double before = base_sh;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (i < N) p[i] = before + x;
        __syncthreads();
        if (tid == 1023) base_sh = before + x;
        __syncthreads();
    }
    const double last = p[N - 1];
    for (int j = tid; j < S; j += 1024) {
        const double target = u[j] * last;
        int64_t lo = 0, hi = N - 1;
        while (lo < hi) {  // first index with CDF > target
            const int64_t mid = (lo + hi) / 2;
            if (p[mid] > target)
                hi = mid;
            else
                lo = mid + 1;
        }
        const double pq = (p[lo] - (lo > 0 ? p[lo - 1] : 0.0)) / last;
        q_idx[j] = (int32_t)lo;
        q_w[j] = 1.0 / ((double)N * (double)S * pq);
    }
}

hipError_t launch_sample(double* p, int64_t N, double mix, const double* u, int S, int32_t* q_idx,
                         double* q_w, int64_t nk, hipStream_t s) {
    if (nk <= 0) return hipSuccess;
    if (nk > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sample_kernel, dim3((unsigned)nk), dim3(1024), 0, s, p, N, mix, u, S, q_idx,
                       q_w);
    return hipGetLastError();
}

}  // namespace phx
