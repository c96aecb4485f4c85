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
#include "stage2_lp_tile.hpp"

namespace phx {

static inline int gridn(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535 * 16) g = 65535 * 16;
    if (g < 1) g = 1;
    return (int)g;
}

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
// One-system launch of the fused rate tile: work-group (q tile, state).
// ---------------------------------------------------------------------------
template <int PREC, int TQ, int TN>
__global__ __launch_bounds__(256, 2) void stage2_rates_lp_kernel(RateArgsLP a) {
    extern __shared__ char smem_raw[];
    __shared__ LpShared sh;
    stage2_lp_tile<PREC, TQ, TN>(a, blockIdx.y, blockIdx.x, smem_raw, sh);
}

size_t stage2_lp_lds(int prec, int tq, int rmax, int rp_pad, int nc_pad, int nm, int nW,
                     bool stage) {
    const int BQ = 16 * tq, CQ = 4 * tq, W = 2 * rmax + 1;
    size_t shm = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)rp_pad * sizeof(int);
    shm = (shm + 15) & ~(size_t)15;
    shm += (size_t)CQ * nc_pad * sizeof(cf) + (size_t)CQ * kMBLP * nm * sizeof(cf);
    // staged U_{k+q} rows [CQ][MB][nW] and E_q [CQ][nm][nm]
    if (stage) shm += (size_t)CQ * kMBLP * nW * sizeof(cf) + (size_t)CQ * nm * nm * sizeof(cf);
    shm = (shm + 15) & ~(size_t)15;
    // split-BF16: two buffers of NP pieces x (re, im) x TQ x 64 lanes x 8 BF16
    const int np = prec == PHOEBE_BF16X3 ? 2 : (prec == PHOEBE_BF16X6 ? 3 : 0);
    shm += (size_t)2 * np * 2 * tq * 64 * 16;
    return shm;
}

bool lp_stage_pays(const void* kern, size_t shm0, size_t shm1) {
    if (shm1 > 160 * 1024 - 1024) return false;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm1) !=
        hipSuccess)
        return false;
    int n0 = 0, n1 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n0, kern, 256, shm0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n1, kern, 256, shm1) != hipSuccess)
        return false;
    return n1 >= n0;
}

template <int PREC, int TQ, int TN>
static hipError_t go_stage2_lp(const RateArgsLP& a0, int nst, hipStream_t s) {
    const void* kern = (const void*)stage2_rates_lp_kernel<PREC, TQ, TN>;
    const size_t shm0 = stage2_lp_lds(PREC, TQ, a0.rmax, a0.rp_pad, a0.nc_pad, a0.nm, a0.nW, false);
    const size_t shm1 = stage2_lp_lds(PREC, TQ, a0.rmax, a0.rp_pad, a0.nc_pad, a0.nm, a0.nW, true);
    if (shm0 > 160 * 1024 - 1024) return hipErrorInvalidValue;
    RateArgsLP a = a0;
    a.stage = lp_stage_pays(kern, shm0, shm1) ? 1 : 0;
    const size_t shm = a.stage ? shm1 : shm0;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
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
    // wider tiles in FP32 only: the split-BF16 fragments of TN >= 12 do not fit in registers
    if constexpr (PREC == PHOEBE_FP32) {
        PHX_CASE(1, 12) PHX_CASE(1, 16)
    }
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
                                   int nm, int nW, cf* __restrict__ F, int64_t ldf) {
    const int64_t nc = (int64_t)nm * nW * nW;
    const int64_t total = (int64_t)n_rp * nc;
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
        const int64_t r = t / nc;
        F[r * ldf + (t - r * nc)] = cf{ar, ai};
    }
}

hipError_t launch_fold_all_lp(const cf* G, const cd* U, int n_rp, int nm, int nW, cf* F,
                              hipStream_t s, int64_t ldf) {
    const int64_t nc = (int64_t)nm * nW * nW;
    if (ldf < 0) ldf = nc;
    if (ldf < nc) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fold_all_lp_kernel, dim3(gridn((int64_t)n_rp * nc, 256)), dim3(256), 0, s,
                       G, U, n_rp, nm, nW, F, ldf);
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
