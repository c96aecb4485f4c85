// Reduced-precision forms of the phase and rotation contractions.
//
//   FP32:   operands rounded to FP32, v_mfma_f32_16x16x4f32, FP32 accumulation.
//   BF16x3: FP32 operands split x = hi + lo (two BF16 pieces); products
//           hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16, FP32 accumulation.
//   BF16x6: three pieces hi + lo + lo2; the six products of combined order <= 2.
//
// Phases are formed in FP64 (exact integer reduction of the mesh phase) and then
// rounded.  Band structure, occupations, Gaussians and the rate accumulation
// stay FP64.  MFMA layouts (f32 16x16x4): lane l holds A[l%16][l/16],
// B[l/16][l%16]; (bf16 16x16x32): lane l holds A[l%16][8(l/16)+j],
// B[8(l/16)+j][l%16], j = 0..7; both return row 4(l/16)+v, column l%16.
#include <type_traits>

#include "kernels.hpp"
#include "lowp.hpp"

namespace phx {

static inline int gridn(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535 * 16) g = 65535 * 16;
    if (g < 1) g = 1;
    return (int)g;
}

// ---------------------------------------------------------------------------
// BF16 splitting (round to nearest even on the bit pattern)
// ---------------------------------------------------------------------------
__device__ inline uint16_t bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    const uint32_t r = ((u >> 16) & 1u) + 0x7FFFu;
    return (uint16_t)((u + r) >> 16);
}
__device__ inline float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// pieces of x: NP = 2 (hi, lo) or 3 (hi, lo, lo2)
template <int NP>
__device__ inline void split_bf16(float x, uint16_t* p) {
    float r = x;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        p[i] = bf16_rne(r);
        r = r - bf16_to_f(p[i]);
    }
}

typedef short s8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

__device__ inline f4 mfma_bf16(const s8v& a, const s8v& b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a),
                                                   __builtin_bit_cast(bf8v, b), c, 0, 0, 0);
}

// products of pieces kept for each mode: (piece of A, piece of B)
template <int PREC>
struct Pairs;
template <>
struct Pairs<PHOEBE_BF16X3> {
    static constexpr int NP = 2, N = 3;
    __device__ static constexpr int a(int i) { return i == 2 ? 1 : 0; }
    __device__ static constexpr int b(int i) { return i == 1 ? 1 : 0; }
};
template <>
struct Pairs<PHOEBE_BF16X6> {
    static constexpr int NP = 3, N = 6;
    // (0,0) (0,1) (1,0) (0,2) (1,1) (2,0)
    __device__ static constexpr int a(int i) { return i < 2 ? 0 : (i == 2 ? 1 : (i == 3 ? 0 : (i == 4 ? 1 : 2))); }
    __device__ static constexpr int b(int i) { return i == 0 ? 0 : (i == 1 ? 1 : (i == 2 ? 0 : (i == 3 ? 2 : (i == 4 ? 1 : 0)))); }
};

// ---------------------------------------------------------------------------
// Stage 1 / generic complex GEMM with FP32 output: C[M, N] (cf) = A[M, K] (cd) B[K, N].
// B is cd (g(Re,Rp)) or cf.  Work-group = 4 waves along N, each TM x TN tiles.
// ---------------------------------------------------------------------------
template <class TB>
__device__ inline cf load_cf(const TB* p);
template <>
__device__ inline cf load_cf<cd>(const cd* p) {
    const cd v = *p;
    return cf{(float)v.x, (float)v.y};
}
template <>
__device__ inline cf load_cf<cf>(const cf* p) { return *p; }

template <int TM, int TN, class TB>
__global__ __launch_bounds__(256) void cgemm_f32_kernel(const cd* __restrict__ A, int64_t lda,
                                                        const TB* __restrict__ B, int64_t ldb,
                                                        cf* __restrict__ C, int64_t ldc, int64_t M,
                                                        int64_t N, int K) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * (16 * TM);
    const int64_t n0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * TN);
    if (n0 >= N) return;
    f4 cr[TM][TN], ci[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            cr[i][j] = f4{0, 0, 0, 0};
            ci[i][j] = f4{0, 0, 0, 0};
        }
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + lk;
        cf av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int64_t row = m0 + 16 * i + li;
            av[i] = (row < M && k < K) ? load_cf(A + row * lda + k) : cf{0.f, 0.f};
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t col = n0 + 16 * j + li;
            bv[j] = (col < N && k < K) ? load_cf(B + (int64_t)k * ldb + col) : cf{0.f, 0.f};
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv[j].x, cr[i][j], 0, 0, 0);
                ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv[j].y, ci[i][j], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-av[i].y, bv[j].y, cr[i][j], 0, 0, 0);
                ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].x, ci[i][j], 0, 0, 0);
            }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + 16 * i + 4 * lk + v;
                const int64_t col = n0 + 16 * j + li;
                if (row < M && col < N) C[row * ldc + col] = cf{cr[i][j][v], ci[i][j][v]};
            }
}

// Split-BF16 complex GEMM, K blocks of 32.  Each lane gathers 8 consecutive k of
// its A row and B column, rounds to FP32 and splits into NP pieces.
template <int PREC, int TM, int TN, class TB>
__global__ __launch_bounds__(256, 2) void cgemm_bf16_kernel(const cd* __restrict__ A, int64_t lda,
                                                         const TB* __restrict__ B, int64_t ldb,
                                                         cf* __restrict__ C, int64_t ldc,
                                                         int64_t M, int64_t N, int K) {
    using P = Pairs<PREC>;
    constexpr int NP = P::NP;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * (16 * TM);
    const int64_t n0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * TN);
    if (n0 >= N) return;
    f4 crp[TM][TN], crn[TM][TN], ci[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            crp[i][j] = f4{0, 0, 0, 0};
            crn[i][j] = f4{0, 0, 0, 0};
            ci[i][j] = f4{0, 0, 0, 0};
        }
    for (int k0 = 0; k0 < K; k0 += 32) {
        const int kb = k0 + 8 * lk;
        s8v ar[TM][NP], ai[TM][NP];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int64_t row = m0 + 16 * i + li;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = kb + j;
                const cf v = (row < M && k < K) ? load_cf(A + row * lda + k) : cf{0.f, 0.f};
                uint16_t pr[NP], pi[NP];
                split_bf16<NP>(v.x, pr);
                split_bf16<NP>(v.y, pi);
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    ar[i][p][j] = (short)pr[p];
                    ai[i][p][j] = (short)pi[p];
                }
            }
        }
#pragma unroll
        for (int t = 0; t < TN; ++t) {
            s8v br[NP], bi[NP];
            const int64_t col = n0 + 16 * t + li;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = kb + j;
                const cf v = (col < N && k < K) ? load_cf(B + (int64_t)k * ldb + col) : cf{0.f, 0.f};
                uint16_t pr[NP], pi[NP];
                split_bf16<NP>(v.x, pr);
                split_bf16<NP>(v.y, pi);
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    br[p][j] = (short)pr[p];
                    bi[p][j] = (short)pi[p];
                }
            }
#pragma unroll
            for (int pp = 0; pp < P::N; ++pp) {
                const int pa = P::a(pp), pb = P::b(pp);
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    crp[i][t] = mfma_bf16(ar[i][pa], br[pb], crp[i][t]);
                    crn[i][t] = mfma_bf16(ai[i][pa], bi[pb], crn[i][t]);
                    ci[i][t] = mfma_bf16(ar[i][pa], bi[pb], ci[i][t]);
                    ci[i][t] = mfma_bf16(ai[i][pa], br[pb], ci[i][t]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + 16 * i + 4 * lk + v;
                const int64_t col = n0 + 16 * j + li;
                if (row < M && col < N)
                    C[row * ldc + col] = cf{crp[i][j][v] - crn[i][j][v], ci[i][j][v]};
            }
}

template <class TB>
static hipError_t cgemm_lp(int prec, const cd* A, int64_t lda, const TB* B, int64_t ldb, cf* C,
                           int64_t ldc, int64_t M, int64_t N, int K, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K <= 0) return hipErrorInvalidValue;
    const int TM = M <= 64 ? 4 : 4;
    const int TN = M <= 64 ? 2 : 1;
    dim3 grid((unsigned)((N + 64 * TN - 1) / (64 * TN)), (unsigned)((M + 16 * TM - 1) / (16 * TM)));
    if (grid.y > 65535) return hipErrorInvalidValue;
    if (prec == PHOEBE_FP32) {
        if (TN == 2)
            hipLaunchKernelGGL((cgemm_f32_kernel<4, 2, TB>), grid, dim3(256), 0, s, A, lda, B, ldb,
                               C, ldc, M, N, K);
        else
            hipLaunchKernelGGL((cgemm_f32_kernel<4, 1, TB>), grid, dim3(256), 0, s, A, lda, B, ldb,
                               C, ldc, M, N, K);
    } else if (prec == PHOEBE_BF16X3 || prec == PHOEBE_BF16X6) {
        // one column tile per wave keeps the split fragments within the
        // register budget of two waves per SIMD
        dim3 g1((unsigned)((N + 63) / 64), grid.y);
        if (prec == PHOEBE_BF16X3)
            hipLaunchKernelGGL((cgemm_bf16_kernel<PHOEBE_BF16X3, 4, 1, TB>), g1, dim3(256), 0, s,
                               A, lda, B, ldb, C, ldc, M, N, K);
        else
            hipLaunchKernelGGL((cgemm_bf16_kernel<PHOEBE_BF16X6, 4, 1, TB>), g1, dim3(256), 0, s,
                               A, lda, B, ldb, C, ldc, M, N, K);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cgemm_lp(int prec, const cd* A, int64_t lda, const cd* B, int64_t ldb, cf* C,
                           int64_t ldc, int64_t M, int64_t N, int K, hipStream_t s) {
    return cgemm_lp<cd>(prec, A, lda, B, ldb, C, ldc, M, N, K, s);
}
hipError_t launch_cgemm_lp_cf(int prec, const cd* A, int64_t lda, const cf* B, int64_t ldb, cf* C,
                              int64_t ldc, int64_t M, int64_t N, int K, hipStream_t s) {
    return cgemm_lp<cf>(prec, A, lda, B, ldb, C, ldc, M, N, K, s);
}

// ---------------------------------------------------------------------------
// Fold of the stage-1 result by U_k^dagger (FP32) into the stage-2 operand.
//   FP32:  F[st][r][c]          cf,   r < rp_pad (multiple of 4),  c < nc_pad
//   BF16:  F[st][part][c][r]    uint16 pieces of re then im (2*NP parts),
//          r < rp_pad (multiple of 32)
// ---------------------------------------------------------------------------
template <int NP>
__global__ void fold_uk_lp_kernel(const cf* __restrict__ G, int64_t ldg, const cd* __restrict__ U,
                                  const int32_t* st_row, int row0, const int32_t* st_kmesh,
                                  const int32_t* st_band, int nst, int n_rp, int nm, int nW,
                                  int cw, int rp_pad, int nc_pad, void* __restrict__ Fout) {
    const int64_t per = (int64_t)rp_pad * nc_pad;
    const int64_t total = (int64_t)nst * per;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int st = (int)(t / per);
        const int64_t o = t - st * per;
        int r, c;
        if (NP == 0) {
            r = (int)(o / nc_pad);
            c = (int)(o - (int64_t)r * nc_pad);
        } else {
            c = (int)(o / rp_pad);
            r = (int)(o - (int64_t)c * rp_pad);
        }
        float ar = 0.f, ai = 0.f;
        const int sa = c / cw, b = c - sa * cw;
        if (r < n_rp && sa < nm && b < nW) {
            const int n = st_band[st];
            const cd* Un = U + ((int64_t)st_kmesh[st] * nW + n) * nW;  // eigenvector n
            const cf* Gk = G + (int64_t)(st_row[st] - row0) * ldg + ((int64_t)r * nm + sa) * nW * nW + b;
            for (int a = 0; a < nW; ++a) {
                const cd u = Un[a];
                const cf g = Gk[a * nW];
                const float ur = (float)u.x, ui = (float)u.y;
                ar = fmaf(ur, g.x, fmaf(ui, g.y, ar));
                ai = fmaf(ur, g.y, fmaf(-ui, g.x, ai));
            }
        }
        if (NP == 0) {
            reinterpret_cast<cf*>(Fout)[t] = cf{ar, ai};
        } else {
            uint16_t* F = reinterpret_cast<uint16_t*>(Fout) + (int64_t)st * 2 * NP * per;
            uint16_t pr[NP > 0 ? NP : 1], pi[NP > 0 ? NP : 1];
            split_bf16<NP>(ar, pr);
            split_bf16<NP>(ai, pi);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                F[(int64_t)p * per + o] = pr[p];
                F[(int64_t)(NP + p) * per + o] = pi[p];
            }
        }
    }
}

hipError_t launch_fold_uk_lp(int prec, const cf* G, int64_t ldg, const cd* U,
                             const int32_t* st_row, int row0, const int32_t* st_kmesh,
                             const int32_t* st_band, int nst, int n_rp, int nm, int nW, int cw,
                             int rp_pad, int nc_pad, void* F, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    if (cw < nW || (int64_t)cw * nm > nc_pad) return hipErrorInvalidValue;
    const int g = gridn((int64_t)nst * rp_pad * nc_pad, 256);
    if (prec == PHOEBE_FP32)
        hipLaunchKernelGGL(fold_uk_lp_kernel<0>, dim3(g), dim3(256), 0, s, G, ldg, U, st_row, row0,
                           st_kmesh, st_band, nst, n_rp, nm, nW, cw, rp_pad, nc_pad, F);
    else if (prec == PHOEBE_BF16X3)
        hipLaunchKernelGGL(fold_uk_lp_kernel<2>, dim3(g), dim3(256), 0, s, G, ldg, U, st_row, row0,
                           st_kmesh, st_band, nst, n_rp, nm, nW, cw, rp_pad, nc_pad, F);
    else
        hipLaunchKernelGGL(fold_uk_lp_kernel<3>, dim3(g), dim3(256), 0, s, G, ldg, U, st_row, row0,
                           st_kmesh, st_band, nst, n_rp, nm, nW, cw, rp_pad, nc_pad, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused stage 2 + rotations + rate terms, reduced precision.
// Same work decomposition as the FP64 kernel: one state x 16*TQ q per
// work-group, 4 waves with TN column tiles each.  Accumulator row of lane
// group lg, result v is 4*lg + v; the rotation works in four chunks c = lg
// (tile rows 4c .. 4c+3), in FP32 on the VALU.
// ---------------------------------------------------------------------------
template <int PREC, int TQ, int TN>
__global__ __launch_bounds__(256, 2) void stage2_rates_lp_kernel(RateArgsLP a) {
    constexpr int BQ = 16 * TQ;
    constexpr int CQ = 4 * TQ;
    constexpr int NP = PREC == PHOEBE_BF16X3 ? 2 : (PREC == PHOEBE_BF16X6 ? 3 : 1);
    extern __shared__ char smem_raw[];
    const int W = 2 * a.rmax + 1;
    const int nW = a.nW, nm = a.nm;
    cd* sAx = reinterpret_cast<cd*>(smem_raw);                // [BQ][3][W]
    int* sRp = reinterpret_cast<int*>(sAx + BQ * 3 * W);      // [rp_pad]
    size_t off = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)a.rp_pad * sizeof(int);
    off = (off + 15) & ~(size_t)15;
    cf* sX = reinterpret_cast<cf*>(smem_raw + off);            // [CQ][nc_pad]
    cf* sY = sX + CQ * a.nc_pad;                               // [CQ][MB][nm]
    __shared__ double sRed[4];
    __shared__ int sKq[CQ];
    __shared__ int sQ[CQ];
    __shared__ double sWq[CQ];

    const int st = blockIdx.y;
    const int qt = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int row = a.st_row[st];
    int64_t qbeg = 0, qcount = a.nq_mesh;
    if (a.q_off) {
        qbeg = a.q_off[row];
        qcount = a.q_off[row + 1] - qbeg;
    }
    const int64_t qt0 = (int64_t)qt * BQ;
    if (qt0 >= qcount) {
        if (tid == 0) a.partial[(int64_t)st * a.n_qtiles + qt] = 0.0;
        return;
    }
    const Mesh mesh = a.mesh;
    for (int i = tid; i < BQ * 3 * W; i += 256) {
        const int ql = i / (3 * W);
        const int d = (i / W) % 3;
        const int r = i % W - a.rmax;
        const int64_t j = qt0 + ql;
        cd v = {0.0, 0.0};
        if (j < qcount) {
            const int64_t q = a.q_idx ? (int64_t)a.q_idx[qbeg + j] : j;
            int i0, i1, i2;
            mesh_triple(q, mesh, i0, i1, i2);
            const int id = d == 0 ? i0 : (d == 1 ? i1 : i2);
            const int N = d == 0 ? mesh.n0 : (d == 1 ? mesh.n1 : mesh.n2);
            int t = (id * r) % N;
            if (t < 0) t += N;
            v = expi2pi((double)t / N);
        }
        sAx[i] = v;
    }
    const int zero_packed = a.rmax | (a.rmax << 8) | (a.rmax << 16);
    for (int i = tid; i < a.rp_pad; i += 256) sRp[i] = i < a.n_rp ? a.rp_packed[i] : zero_packed;
    __syncthreads();

    f4 crp[TQ][TN], ci[TQ][TN];
#pragma unroll
    for (int i = 0; i < TQ; ++i)
#pragma unroll
        for (int t = 0; t < TN; ++t) {
            crp[i][t] = f4{0, 0, 0, 0};
            ci[i][t] = f4{0, 0, 0, 0};
        }
    const int colbase = wave * TN * 16 + li;
    if constexpr (PREC == PHOEBE_FP32) {
        const cf* Fst = reinterpret_cast<const cf*>(a.F) + (int64_t)st * a.rp_pad * a.nc_pad;
        const int ldf = a.nc_pad;
        for (int k0 = 0; k0 < a.rp_pad; k0 += 4) {
            const int k = k0 + lg;
            const int pk = sRp[k];
            const int p0 = pk & 255, p1 = (pk >> 8) & 255, p2 = (pk >> 16) & 255;
            cf bv[TN];
            const cf* Fr = Fst + (int64_t)k * ldf + colbase;
#pragma unroll
            for (int t = 0; t < TN; ++t) bv[t] = Fr[t * 16];
            float ar[TQ], ai[TQ];
#pragma unroll
            for (int i = 0; i < TQ; ++i) {
                const cd* ax = sAx + (16 * i + li) * 3 * W;
                const cd ph = cmul(cmul(ax[p0], ax[W + p1]), ax[2 * W + p2]);
                ar[i] = (float)ph.x;
                ai[i] = (float)ph.y;
            }
#pragma unroll
            for (int i = 0; i < TQ; ++i)
#pragma unroll
                for (int t = 0; t < TN; ++t) {
                    crp[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bv[t].x, crp[i][t], 0, 0, 0);
                    ci[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bv[t].y, ci[i][t], 0, 0, 0);
                }
#pragma unroll
            for (int i = 0; i < TQ; ++i)
#pragma unroll
                for (int t = 0; t < TN; ++t) {
                    crp[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[i], bv[t].y, crp[i][t], 0, 0, 0);
                    ci[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], bv[t].x, ci[i][t], 0, 0, 0);
                }
        }
    } else {
        using P = Pairs<PREC>;
        const int64_t per = (int64_t)a.rp_pad * a.nc_pad;
        const uint16_t* Fst = reinterpret_cast<const uint16_t*>(a.F) + (int64_t)st * 2 * NP * per;
        // The A fragments (phase pieces) are the same for the four waves: the
        // work-group forms each once per K step into LDS (double-buffered,
        // [buf][piece][re, im][i][lane] slots of 8 BF16), TPS threads per slot.
        s8v* sAf = reinterpret_cast<s8v*>(sY + CQ * kMBLP * nm);
        constexpr int SLOTS = TQ * 64;
        constexpr int TPS = 256 / SLOTS;  // threads per slot
        constexpr int JPT = 8 / TPS;      // phases per thread
        const int fslot = tid / TPS, fpart = tid % TPS;
        const int fi = fslot / 64, fl = fslot % 64;
        const cd* fax = sAx + (16 * fi + (fl & 15)) * 3 * W;
        int buf = 0;
        for (int k0 = 0; k0 < a.rp_pad; k0 += 32, buf ^= 1) {
            const int kb = k0 + 8 * lg;
            {
                // FP64 product of the three axis factors, rounded to FP32, split
                short* dr = reinterpret_cast<short*>(sAf + ((buf * NP) * 2 * TQ + fi) * 64 + fl);
#pragma unroll
                for (int jj = 0; jj < JPT; ++jj) {
                    const int j = fpart * JPT + jj;
                    const int pk = sRp[k0 + 8 * (fl >> 4) + j];
                    const cd ph = cmul(cmul(fax[pk & 255], fax[W + ((pk >> 8) & 255)]),
                                       fax[2 * W + ((pk >> 16) & 255)]);
                    uint16_t pr[NP], pi[NP];
                    split_bf16<NP>((float)ph.x, pr);
                    split_bf16<NP>((float)ph.y, pi);
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        dr[((p * 2 + 0) * TQ * 64) * 8 + j] = (short)pr[p];
                        dr[((p * 2 + 1) * TQ * 64) * 8 + j] = (short)pi[p];
                    }
                }
            }
            __syncthreads();
            s8v ar[TQ][NP], ai[TQ][NP];
#pragma unroll
            for (int i = 0; i < TQ; ++i)
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    ar[i][p] = sAf[(((buf * NP + p) * 2 + 0) * TQ + i) * 64 + lane];
                    ai[i][p] = sAf[(((buf * NP + p) * 2 + 1) * TQ + i) * 64 + lane];
                }
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                s8v br[NP], bi[NP];
                const int64_t o = (int64_t)(colbase + 16 * t) * a.rp_pad + kb;
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    br[p] = *reinterpret_cast<const s8v*>(Fst + (int64_t)p * per + o);
                    bi[p] = *reinterpret_cast<const s8v*>(Fst + (int64_t)(NP + p) * per + o);
                }
#pragma unroll
                for (int pp = 0; pp < P::N; ++pp) {
                    const int pa = P::a(pp), pb = P::b(pp);
#pragma unroll
                    for (int i = 0; i < TQ; ++i) {
                        const s8v nai = ai[i][pa] ^ (short)0x8000;  // -Im(A): flip the sign bits
                        crp[i][t] = mfma_bf16(ar[i][pa], br[pb], crp[i][t]);
                        crp[i][t] = mfma_bf16(nai, bi[pb], crp[i][t]);
                        ci[i][t] = mfma_bf16(ar[i][pa], bi[pb], ci[i][t]);
                        ci[i][t] = mfma_bf16(ai[i][pa], br[pb], ci[i][t]);
                    }
                }
            }
        }
    }

    // ---- rotations (FP32) and rate terms (FP64) ----
    const int ldf = a.nc_pad;
    const int kmesh = a.st_kmesh[st];
    const int nband = a.st_band[st];
    const int mlo = a.st_mlo[st], mhi = a.st_mhi[st];
    int k0i, k1i, k2i;
    mesh_triple(kmesh, mesh, k0i, k1i, k2i);
    const double eps_n = a.eps[(int64_t)kmesh * nW + nband];
    const double inv_s2 = 1.0 / (a.sigma * a.sigma);
    double gacc = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        __syncthreads();
        if (lg == c) {
#pragma unroll
            for (int i = 0; i < TQ; ++i)
#pragma unroll
                for (int t = 0; t < TN; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        sX[(4 * i + v) * ldf + colbase + t * 16] = cf{crp[i][t][v], ci[i][t][v]};
        }
        if (tid < CQ) {
            const int cc = tid;
            const int qloc = 16 * (cc >> 2) + 4 * c + (cc & 3);
            const int64_t j = qt0 + qloc;
            int kq = -1, q = 0;
            double w = 0.0;
            if (j < qcount) {
                q = a.q_idx ? a.q_idx[qbeg + j] : (int)j;
                w = a.q_w ? a.q_w[qbeg + j] : 1.0;
                int q0, q1, q2;
                mesh_triple(q, mesh, q0, q1, q2);
                kq = (int)mesh_linear((k0i + q0) % mesh.n0, (k1i + q1) % mesh.n1,
                                      (k2i + q2) % mesh.n2, mesh);
            }
            sKq[cc] = kq;
            sQ[cc] = q;
            sWq[cc] = w;
        }
        __syncthreads();
        for (int m0 = mlo; m0 <= mhi; m0 += kMBLP) {
            const int nmb = min(kMBLP, mhi - m0 + 1);
            for (int it = tid; it < CQ * nmb * nm; it += 256) {
                const int cc = it / (nmb * nm);
                const int r = it - cc * nmb * nm;
                const int mb = r / nm, sa = r - mb * nm;
                const int kq = sKq[cc];
                float yr = 0.f, yi = 0.f;
                if (kq >= 0) {
                    const cf* Xr = sX + cc * ldf + sa * nW;
                    const cd* Um = a.U + ((int64_t)kq * nW + m0 + mb) * nW;  // eigenvector m
                    for (int b = 0; b < nW; ++b) {
                        const cf x = Xr[b];
                        const cd u = Um[b];
                        const float ur = (float)u.x, ui = (float)u.y;
                        yr = fmaf(x.x, ur, fmaf(-x.y, ui, yr));
                        yi = fmaf(x.x, ui, fmaf(x.y, ur, yi));
                    }
                }
                sY[(cc * kMBLP + mb) * nm + sa] = cf{yr, yi};
            }
            __syncthreads();
            for (int it = tid; it < CQ * nmb * nm; it += 256) {
                const int cc = it / (nmb * nm);
                const int r = it - cc * nmb * nm;
                const int mb = r / nm, nu = r - mb * nm;
                const int kq = sKq[cc];
                if (kq < 0) continue;
                const int64_t q = sQ[cc];
                const cf* Yr = sY + (cc * kMBLP + mb) * nm;
                const cd* Eq = a.E + (q * nm + nu) * nm;
                float zr = 0.f, zi = 0.f;
                for (int sa = 0; sa < nm; ++sa) {
                    const cd e = Eq[sa];
                    const float er = (float)e.x, ei = (float)e.y;
                    const cf y = Yr[sa];
                    zr = fmaf(er, y.x, fmaf(-ei, y.y, zr));
                    zi = fmaf(er, y.y, fmaf(ei, y.x, zi));
                }
                const int m = m0 + mb;
                const double x = eps_n - a.eps[(int64_t)kq * nW + m];
                const double fm = a.focc[(int64_t)kq * nW + m];
                const double w = a.omega[q * nm + nu], nbq = a.nb[q * nm + nu];
                const double y1 = x - w, y2 = x + w;
                const double g1 = exp(-y1 * y1 * inv_s2), g2 = exp(-y2 * y2 * inv_s2);
                const double z2 = (double)zr * zr + (double)zi * zi;
                gacc += sWq[cc] * z2 * ((nbq + 1.0 - fm) * g1 + (nbq + fm) * g2);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) gacc += __shfl_xor(gacc, o, 64);
    if (lane == 0) sRed[wave] = gacc;
    __syncthreads();
    if (tid == 0)
        a.partial[(int64_t)st * a.n_qtiles + qt] = (sRed[0] + sRed[1]) + (sRed[2] + sRed[3]);
}

size_t stage2_lp_lds(int prec, int tq, int rmax, int rp_pad, int nc_pad, int nm) {
    const int BQ = 16 * tq, CQ = 4 * tq, W = 2 * rmax + 1;
    size_t shm = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)rp_pad * sizeof(int);
    shm = (shm + 15) & ~(size_t)15;
    shm += (size_t)CQ * nc_pad * sizeof(cf) + (size_t)CQ * kMBLP * nm * sizeof(cf);
    shm = (shm + 15) & ~(size_t)15;
    // split-BF16: two buffers of NP pieces x (re, im) x TQ x 64 lanes x 8 BF16
    const int np = prec == PHOEBE_BF16X3 ? 2 : (prec == PHOEBE_BF16X6 ? 3 : 0);
    shm += (size_t)2 * np * 2 * tq * 64 * 16;
    return shm;
}

template <int PREC, int TQ, int TN>
static hipError_t go_stage2_lp(const RateArgsLP& a, int nst, hipStream_t s) {
    const size_t shm = stage2_lp_lds(PREC, TQ, a.rmax, a.rp_pad, a.nc_pad, a.nm);
    if (shm > 160 * 1024 - 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)stage2_rates_lp_kernel<PREC, TQ, TN>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    const size_t fbytes = (PREC == PHOEBE_FP32 ? sizeof(cf)
                                               : (PREC == PHOEBE_BF16X3 ? 4 : 6) * sizeof(uint16_t)) *
                          (size_t)a.rp_pad * a.nc_pad;
    for (int s0 = 0; s0 < nst; s0 += 65535) {
        const int ns = nst - s0 < 65535 ? nst - s0 : 65535;
        RateArgsLP b = a;
        b.F = reinterpret_cast<const char*>(a.F) + (size_t)s0 * fbytes;
        b.st_kmesh += s0;
        b.st_band += s0;
        b.st_row += s0;
        b.st_mlo += s0;
        b.st_mhi += s0;
        b.partial = a.partial + (int64_t)s0 * a.n_qtiles;
        hipLaunchKernelGGL((stage2_rates_lp_kernel<PREC, TQ, TN>), dim3(a.n_qtiles, ns), dim3(256),
                           shm, s, b);
    }
    return hipGetLastError();
}

template <int PREC>
static hipError_t dispatch_lp(const RateArgsLP& a, int nst, int tq, int tn, hipStream_t s) {
#define PHX_CASE(TQv, TNv) \
    if (tq == TQv && tn == TNv) return go_stage2_lp<PREC, TQv, TNv>(a, nst, s);
    PHX_CASE(2, 1) PHX_CASE(2, 2) PHX_CASE(2, 3) PHX_CASE(2, 4) PHX_CASE(1, 6) PHX_CASE(1, 8)
#undef PHX_CASE
    return hipErrorInvalidValue;
}

int stage2_lp_config(int nm, int nW, int* tq_out, int* tn_out) {
    const int nc_pad = stage2_config(nm, nW, tq_out, tn_out);
    if (*tq_out > 2) *tq_out = 2;  // keeps the split-BF16 fragments in registers
    return nc_pad;
}

hipError_t launch_stage2_rates_lp(int prec, const RateArgsLP& a, int nst, hipStream_t s) {
    if (nst <= 0 || a.n_qtiles <= 0) return hipSuccess;
    int tq = 0, tn = 0;
    if (stage2_lp_config(a.nm, a.nW, &tq, &tn) != a.nc_pad) return hipErrorInvalidValue;
    if (prec == PHOEBE_FP32) return dispatch_lp<PHOEBE_FP32>(a, nst, tq, tn, s);
    if (prec == PHOEBE_BF16X3) return dispatch_lp<PHOEBE_BF16X3>(a, nst, tq, tn, s);
    if (prec == PHOEBE_BF16X6) return dispatch_lp<PHOEBE_BF16X6>(a, nst, tq, tn, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// interp_g in reduced precision: fold (all bands) and rotation in FP32.
// ---------------------------------------------------------------------------
__global__ void fold_all_lp_kernel(const cf* __restrict__ G, const cd* __restrict__ U, int n_rp,
                                   int nm, int nW, cf* __restrict__ F) {
    const int64_t total = (int64_t)n_rp * nm * nW * nW;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nW);
        const int n = (int)((t / nW) % nW);
        const int64_t rs = t / ((int64_t)nW * nW);
        const cf* Gp = G + rs * nW * nW + b;
        float ar = 0.f, ai = 0.f;
        for (int a = 0; a < nW; ++a) {
            const cd u = U[a * nW + n];
            const cf g = Gp[a * nW];
            const float ur = (float)u.x, ui = (float)u.y;
            ar = fmaf(ur, g.x, fmaf(ui, g.y, ar));
            ai = fmaf(ur, g.y, fmaf(-ui, g.x, ai));
        }
        F[t] = cf{ar, ai};
    }
}

hipError_t launch_fold_all_lp(const cf* G, const cd* U, int n_rp, int nm, int nW, cf* F,
                              hipStream_t s) {
    hipLaunchKernelGGL(fold_all_lp_kernel, dim3(gridn((int64_t)n_rp * nm * nW * nW, 256)),
                       dim3(256), 0, s, G, U, n_rp, nm, nW, F);
    return hipGetLastError();
}

__global__ void rotate_g_lp_kernel(const cf* __restrict__ X, int64_t nq, const cd* __restrict__ Ukq,
                                   const cd* __restrict__ E, int nW, int nm, cd* __restrict__ g) {
    const int64_t total = nq * nW * nW;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(t % nW);
        const int n = (int)((t / nW) % nW);
        const int64_t q = t / ((int64_t)nW * nW);
        const cf* Xq = X + q * nm * nW * nW;
        const cd* Uq = Ukq + q * nW * nW;
        const cd* Eq = E + q * nm * nm;
        float yr[32], yi[32];
        for (int sa = 0; sa < nm; ++sa) {
            float ar = 0.f, ai = 0.f;
            const cf* xr = Xq + ((int64_t)sa * nW + n) * nW;
            for (int b = 0; b < nW; ++b) {
                const cf x = xr[b];
                const cd u = Uq[b * nW + m];
                const float ur = (float)u.x, ui = (float)u.y;
                ar = fmaf(x.x, ur, fmaf(-x.y, ui, ar));
                ai = fmaf(x.x, ui, fmaf(x.y, ur, ai));
            }
            yr[sa] = ar;
            yi[sa] = ai;
        }
        cd* go = g + q * nm * nW * nW;
        for (int nu = 0; nu < nm; ++nu) {
            float zr = 0.f, zi = 0.f;
            for (int sa = 0; sa < nm; ++sa) {
                const cd e = Eq[nu * nm + sa];
                const float er = (float)e.x, ei = (float)e.y;
                zr = fmaf(er, yr[sa], fmaf(-ei, yi[sa], zr));
                zi = fmaf(er, yi[sa], fmaf(ei, yr[sa], zi));
            }
            go[((int64_t)nu * nW + n) * nW + m] = cd{(double)zr, (double)zi};
        }
    }
}

// The same rotation with one work-group per q (nW <= 16): X[q] and E_q (rounded
// to FP32) staged in LDS once; thread (n, m) holds U_{k+q}[:, m] and Y[sa] in
// registers.  The sums run in the same order as above.
template <int NMX>
__global__ __launch_bounds__(256) void rotate_g_lp_lds_kernel(const cf* __restrict__ X,
                                                              const cd* __restrict__ Ukq,
                                                              const cd* __restrict__ E, int nW,
                                                              int nm, cd* __restrict__ g) {
    extern __shared__ char smem_raw[];
    const int nc = nm * nW * nW;
    cf* sX = reinterpret_cast<cf*>(smem_raw);  // [nm][nW][nW]
    cf* sE = sX + nc;                          // [nu][sa]
    const int64_t q = blockIdx.x;
    const int tid = threadIdx.x;
    const cf* Xq = X + q * nc;
    for (int i = tid; i < nc; i += blockDim.x) sX[i] = Xq[i];
    const cd* Eq = E + q * nm * nm;
    for (int i = tid; i < nm * nm; i += blockDim.x) sE[i] = cf{(float)Eq[i].x, (float)Eq[i].y};
    __syncthreads();
    if (tid >= nW * nW) return;
    const int n = tid / nW, m = tid - n * nW;
    const cd* Uq = Ukq + q * nW * nW;
    float ur[16], ui[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        const cd u = b < nW ? Uq[b * nW + m] : cd{0.0, 0.0};
        ur[b] = (float)u.x;
        ui[b] = (float)u.y;
    }
    float yr[NMX], yi[NMX];
#pragma unroll
    for (int sa = 0; sa < NMX; ++sa) {
        float ar = 0.f, ai = 0.f;
        if (sa < nm) {
            const cf* xr = sX + (sa * nW + n) * nW;
#pragma unroll
            for (int b = 0; b < 16; ++b)
                if (b < nW) {
                    const cf x = xr[b];
                    ar = fmaf(x.x, ur[b], fmaf(-x.y, ui[b], ar));
                    ai = fmaf(x.x, ui[b], fmaf(x.y, ur[b], ai));
                }
        }
        yr[sa] = ar;
        yi[sa] = ai;
    }
    cd* go = g + q * nc + n * nW + m;
    for (int nu = 0; nu < nm; ++nu) {
        const cf* er = sE + nu * nm;
        float zr = 0.f, zi = 0.f;
#pragma unroll
        for (int sa = 0; sa < NMX; ++sa)
            if (sa < nm) {
                zr = fmaf(er[sa].x, yr[sa], fmaf(-er[sa].y, yi[sa], zr));
                zi = fmaf(er[sa].x, yi[sa], fmaf(er[sa].y, yr[sa], zi));
            }
        go[(int64_t)nu * nW * nW] = cd{(double)zr, (double)zi};
    }
}

hipError_t launch_rotate_g_lp(const cf* X, int64_t nq, const cd* Ukq, const cd* E, int nW, int nm,
                              cd* g, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    const size_t shm = ((size_t)nm * nW * nW + (size_t)nm * nm) * sizeof(cf);
    if (nW <= 16 && nm <= 32 && shm <= 160 * 1024 && nq <= 2147483647LL) {
        const int block = (nW * nW + 63) / 64 * 64 < 64 ? 64 : (nW * nW + 63) / 64 * 64;
        auto go = [&](auto nmx) {
            constexpr int NMX = decltype(nmx)::value;
            hipError_t e = hipFuncSetAttribute((const void*)rotate_g_lp_lds_kernel<NMX>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(rotate_g_lp_lds_kernel<NMX>, dim3((unsigned)nq), dim3(block), shm, s,
                               X, Ukq, E, nW, nm, g);
            return hipGetLastError();
        };
        if (nm <= 8) return go(std::integral_constant<int, 8>{});
        if (nm <= 16) return go(std::integral_constant<int, 16>{});
        return go(std::integral_constant<int, 32>{});
    }
    hipLaunchKernelGGL(rotate_g_lp_kernel, dim3(gridn(nq * nW * nW, 128)), dim3(128), 0, s, X, nq,
                       Ukq, E, nW, nm, g);
    return hipGetLastError();
}

}  // namespace phx
