// Dense building blocks on gfx950: phase tables, complex FP64 GEMM on MFMA,
// batched Hermitian Jacobi eigensolver, phonon/electron post-processing and
// mesh bookkeeping (window, ordered compaction).
#include "kernels.hpp"

namespace phx {

// ---------------------------------------------------------------------------
// Phase table P[p, r] = e^{i 2 pi x_p . R_r}
// Mesh points use exact integer reduction: x.R = sum_d (i_d R_d mod N_d)/N_d.
// Fractional points reduce x.R by its nearest integer before sincospi.
// ---------------------------------------------------------------------------
__global__ void phase_table_kernel(const double* frac, const int32_t* idx, Mesh m, int64_t np,
                                   const int32_t* R, int nR, cd* P, int64_t ldp) {
    const int64_t total = np * (int64_t)nR;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = t / nR;
        const int r = (int)(t - p * nR);
        const int r0 = R[3 * r], r1 = R[3 * r + 1], r2 = R[3 * r + 2];
        double x;
        if (frac) {
            const double* f = frac + 3 * p;
            x = f[0] * r0 + f[1] * r1 + f[2] * r2;
            x -= rint(x);
        } else {
            const int64_t li = idx ? (int64_t)idx[p] : p;
            int i0, i1, i2;
            mesh_triple(li, m, i0, i1, i2);
            int a0 = (int)(((int64_t)i0 * r0) % m.n0);
            int a1 = (int)(((int64_t)i1 * r1) % m.n1);
            int a2 = (int)(((int64_t)i2 * r2) % m.n2);
            if (a0 < 0) a0 += m.n0;
            if (a1 < 0) a1 += m.n1;
            if (a2 < 0) a2 += m.n2;
            x = (double)a0 / m.n0 + (double)a1 / m.n1 + (double)a2 / m.n2;
            x -= rint(x);
        }
        P[p * ldp + r] = expi2pi(x);
    }
}

static inline int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535 * 16) g = 65535 * 16;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_phase_table(const double* frac, const int32_t* idx, Mesh m, int64_t np,
                              const int32_t* R, int nR, cd* P, int64_t ldp, hipStream_t s) {
    if (np <= 0 || nR <= 0) return hipSuccess;
    hipLaunchKernelGGL(phase_table_kernel, dim3(grid_for(np * nR, 256)), dim3(256), 0, s, frac,
                       idx, m, np, R, nR, P, ldp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Complex FP64 GEMM C = A B on v_mfma_f64_16x16x4f64.
// A work-group is 4 waves side by side along N; each wave owns TM x TN tiles
// of 16 x 16.  MFMA operand layouts (16x16x4 f64): lane l holds A[l%16][l/16],
// B[l/16][l%16]; result v (0..3) of lane l is D[l/16 + 4v][l%16].
// Complex product with 4 real MFMAs: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
// ---------------------------------------------------------------------------
template <int TM, int TN>
__global__ __launch_bounds__(256, 2) void zgemm_kernel(const cd* __restrict__ A, int64_t lda,
                                                    const cd* __restrict__ B, int64_t ldb,
                                                    cd* __restrict__ C, int64_t ldc, int64_t M,
                                                    int64_t N, int K) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * (16 * TM);
    const int64_t n0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * TN);
    if (n0 >= N) return;
    d4 cr[TM][TN], ci[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            cr[i][j] = d4{0, 0, 0, 0};
            ci[i][j] = d4{0, 0, 0, 0};
        }
    cd a_cur[TM], b_cur[TN];
    auto load = [&](int k0, cd* av, cd* bv) {
        const int k = k0 + lk;
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int64_t row = m0 + 16 * i + li;
            av[i] = (row < M && k < K) ? A[row * lda + k] : cd{0.0, 0.0};
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t col = n0 + 16 * j + li;
            bv[j] = (col < N && k < K) ? B[(int64_t)k * ldb + col] : cd{0.0, 0.0};
        }
    };
    // operands are prefetched two k-steps ahead: one step of MFMA work is
    // shorter than the HBM latency of the streamed B operand
    cd a_n1[TM], b_n1[TN];
    load(0, a_cur, b_cur);
    load(4, a_n1, b_n1);  // zeros where k >= K
    for (int k0 = 0; k0 < K; k0 += 4) {
        cd a_n2[TM], b_n2[TN];
        load(k0 + 8, a_n2, b_n2);  // zeros past K
        // two passes over the tiles, so that dependent MFMAs on one accumulator
        // are 2 TM TN - 1 instructions apart
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_cur[i].x, b_cur[j].x, cr[i][j], 0, 0, 0);
                ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_cur[i].x, b_cur[j].y, ci[i][j], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_cur[i].y, b_cur[j].y, cr[i][j], 0, 0, 0);
                ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_cur[i].y, b_cur[j].x, ci[i][j], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            a_cur[i] = a_n1[i];
            a_n1[i] = a_n2[i];
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            b_cur[j] = b_n1[j];
            b_n1[j] = b_n2[j];
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = m0 + 16 * i + lk + 4 * v;
                const int64_t col = n0 + 16 * j + li;
                if (row < M && col < N) C[row * ldc + col] = cd{cr[i][j][v], ci[i][j][v]};
            }
}

hipError_t launch_zgemm(const cd* A, int64_t lda, const cd* B, int64_t ldb, cd* C, int64_t ldc,
                        int64_t M, int64_t N, int K, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K <= 0) return hipErrorInvalidValue;
    // Tall-and-narrow products (Fourier transforms over many points) use 4 row
    // tiles per wave; short-and-wide ones (stage 1, M = a batch of k) cover all
    // rows of up to 128 in one work-group so each B column is read once.
    if (M <= 64) {
        const int TM = 4, TN = 2;
        dim3 grid((unsigned)((N + 4 * 16 * TN - 1) / (4 * 16 * TN)), (unsigned)((M + 63) / 64));
        hipLaunchKernelGGL((zgemm_kernel<TM, TN>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                           M, N, K);
    } else if (M <= 128) {
        const int TM = 8, TN = 1;
        dim3 grid((unsigned)((N + 4 * 16 * TN - 1) / (4 * 16 * TN)), (unsigned)((M + 127) / 128));
        hipLaunchKernelGGL((zgemm_kernel<TM, TN>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                           M, N, K);
    } else {
        const int TM = 4, TN = 1;
        dim3 grid((unsigned)((N + 4 * 16 * TN - 1) / (4 * 16 * TN)),
                  (unsigned)((M + 16 * TM - 1) / (16 * TM)));
        hipLaunchKernelGGL((zgemm_kernel<TM, TN>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                           M, N, K);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// In-place transpose of a batch of n x n matrices: the rate path keeps each
// eigenvector contiguous (Ut[k, band, orbital] = U_k[orbital, band]), so a
// band's column is one coalesced read.
// ---------------------------------------------------------------------------
__global__ void transpose_batch_kernel(cd* U, int64_t count, int n) {
    const int64_t total = count * n * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(t % n);
        const int i = (int)((t / n) % n);
        if (i >= j) continue;
        const int64_t base = (t / ((int64_t)n * n)) * n * n;
        const cd a = U[base + (int64_t)i * n + j];
        U[base + (int64_t)i * n + j] = U[base + (int64_t)j * n + i];
        U[base + (int64_t)j * n + i] = a;
    }
}

hipError_t launch_transpose_batch(cd* U, int64_t count, int n, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(transpose_batch_kernel, dim3(grid_for(count * n * n, 256)), dim3(256), 0, s,
                       U, count, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Mass weighting of the force constants: D-kernel entries Phi(R)/sqrt(M_s M_s')
// ---------------------------------------------------------------------------
__global__ void mass_weight_kernel(const double* phi, const double* mass, int nR, int nm, cd* out) {
    const int64_t total = (int64_t)nR * nm * nm;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(t % nm);
        const int i = (int)((t / nm) % nm);
        out[t] = cd{phi[t] / sqrt(mass[i / 3] * mass[j / 3]), 0.0};
    }
}

hipError_t launch_mass_weight(const double* phi, const double* mass, int nR, int nm, cd* out,
                              hipStream_t s) {
    hipLaunchKernelGGL(mass_weight_kernel, dim3(grid_for((int64_t)nR * nm * nm, 256)), dim3(256),
                       0, s, phi, mass, nR, nm, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched Hermitian eigensolver: cyclic Jacobi with the round-robin parallel
// ordering, one wavefront per matrix, matrix and eigenvectors in LDS.
// Rotation of pivot (p, q) with a = A_pp, d = A_qq, b = A_pq = |b| e^{i phi}:
//   tau = (d - a) / (2|b|), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1/sqrt(1 + t^2), s = t c,
//   J_pp = J_qq = c, J_pq = s e^{i phi}, J_qp = -s e^{-i phi};  A <- J^H A J, V <- V J.
// ---------------------------------------------------------------------------
__device__ inline void rr_pair(int k, int round, int np, int& p, int& q) {
    const int m = np - 1;
    int a, b;
    if (k == 0) {
        a = m;
        b = round;
    } else {
        a = (round + k) % m;
        b = (round - k + m) % m;
    }
    p = a < b ? a : b;
    q = a < b ? b : a;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// NT > 0 fixes the matrix order at compile time (index arithmetic without
// integer division); NT = 0 takes it from the argument.
template <int NT>
__global__ __launch_bounds__(64) void eig_herm_kernel(cd* __restrict__ Aall, int n_arg,
                                                      double* __restrict__ w_out,
                                                      cd* __restrict__ V_out) {
    const int n = NT > 0 ? NT : n_arg;
    extern __shared__ char smem_raw[];
    cd* A = reinterpret_cast<cd*>(smem_raw);
    // odd row stride: 16 lanes walking down a column of 16-byte elements hit 16
    // distinct 4-bank groups (an even stride such as 16 would serialise them)
    const int ld = n | 1;
    cd* V = A + n * ld;
    double* rc = reinterpret_cast<double*>(V + n * ld);  // [n/2+1] c
    double* rs = rc + (n / 2 + 1);                         // s
    cd* re = reinterpret_cast<cd*>(rs + (n / 2 + 1));      // e^{i phi}
    int* rp = reinterpret_cast<int*>(re + (n / 2 + 1));    // p
    int* rq = rp + (n / 2 + 1);                            // q
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x;
    cd* Ag = Aall + b * (int64_t)n * n;
    for (int i = lane; i < n * n; i += 64) {
        const int r = i / n, c = i % n;
        A[r * ld + c] = Ag[i];
        V[r * ld + c] = cd{r == c ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    const int np = n + (n & 1);
    const int half = np / 2;
    const double eps2 = 4.9e-32;  // (2.2e-16)^2
    for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
        int rotated = 0;
        double off = 0.0, dia = 0.0;
        for (int i = lane; i < n * n; i += 64) {
            const int r = i / n, c = i % n;
            const double v = cabs2(A[r * ld + c]);
            if (r == c)
                dia += v;
            else
                off += v;
        }
        off = wave_sum(off);
        dia = wave_sum(dia);
        if (!(off > 1e-32 * dia)) break;
        // A pair is left alone once |A_pq|^2 is at the rounding level of its own diagonal
        // entries or of the mean squared diagonal entry, whichever is larger: with the
        // first test alone, pairs next to a zero eigenvalue keep rotating on rounding noise
        // and the off-diagonal norm never falls below the stopping level above.
        const double skip_abs = eps2 * dia / n;
        for (int round = 0; round < np - 1; ++round) {
            if (lane < half) {
                int p, q;
                rr_pair(lane, round, np, p, q);
                double c = 1.0, s = 0.0;
                cd e = {1.0, 0.0};
                if (q < n) {
                    const double a = A[p * ld + p].x, d = A[q * ld + q].x;
                    const cd bpq = A[p * ld + q];
                    const double bb2 = cabs2(bpq);
                    if (bb2 > fmax(eps2 * fabs(a * d), skip_abs) && bb2 > 0.0) {
                        rotated = 1;
                        // (one reciprocal square root for 1/|b|, one for c: two
                        // divisions and a square root fewer on the round's critical path)
                        const double ib = rsqrt(bb2);
                        const double tau = (d - a) * (0.5 * ib);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(fma(tau, tau, 1.0)));
                        c = rsqrt(fma(t, t, 1.0));
                        s = t * c;
                        e = cd{bpq.x * ib, bpq.y * ib};
                    }
                }
                rc[lane] = c;
                rs[lane] = s;
                re[lane] = e;
                rp[lane] = p;
                rq[lane] = q < n ? q : -1;
            }
            __syncthreads();
            // rows: A'_pj = c A_pj - s e A_qj ; A'_qj = s conj(e) A_pj + c A_qj
            for (int it = lane; it < half * n; it += 64) {
                const int k = it / n, j = it % n;
                const int q = rq[k];
                if (q < 0 || rs[k] == 0.0) continue;
                const int p = rp[k];
                const double c = rc[k], s = rs[k];
                const cd e = re[k];
                const cd apj = A[p * ld + j], aqj = A[q * ld + j];
                const cd eq = cmul(e, aqj);
                const cd ep = cmulc(e, apj);
                A[p * ld + j] = cd{c * apj.x - s * eq.x, c * apj.y - s * eq.y};
                A[q * ld + j] = cd{s * ep.x + c * aqj.x, s * ep.y + c * aqj.y};
            }
            __syncthreads();
            // columns: A'_ip = c A_ip - s conj(e) A_iq ; A'_iq = s e A_ip + c A_iq ; same for V
            for (int it = lane; it < 2 * half * n; it += 64) {
                const int which = it / (half * n);
                const int r = it % (half * n);
                const int k = r / n, i = r % n;
                const int q = rq[k];
                if (q < 0 || rs[k] == 0.0) continue;
                const int p = rp[k];
                const double c = rc[k], s = rs[k];
                const cd e = re[k];
                cd* M = which ? V : A;
                const cd aip = M[i * ld + p], aiq = M[i * ld + q];
                const cd eq = cmulc(e, aiq);
                const cd ep = cmul(e, aip);
                M[i * ld + p] = cd{c * aip.x - s * eq.x, c * aip.y - s * eq.y};
                M[i * ld + q] = cd{s * ep.x + c * aiq.x, s * ep.y + c * aiq.y};
            }
            __syncthreads();
            if (lane < half) {
                const int q = rq[lane];
                if (q >= 0 && rs[lane] != 0.0) {
                    const int p = rp[lane];
                    A[p * ld + q] = cd{0.0, 0.0};
                    A[q * ld + p] = cd{0.0, 0.0};
                    A[p * ld + p].y = 0.0;
                    A[q * ld + q].y = 0.0;
                }
            }
            __syncthreads();
        }
        if (!__any(rotated)) break;  // a sweep with no rotation leaves A unchanged
    }
    // ascending order, ties by index
    for (int i = lane; i < n; i += 64) {
        const double wi = A[i * ld + i].x;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double wj = A[j * ld + j].x;
            rank += (wj < wi) || (wj == wi && j < i);
        }
        w_out[b * n + rank] = wi;
        cd* Vg = V_out + b * (int64_t)n * n;
        for (int r = 0; r < n; ++r) Vg[r * n + rank] = V[r * ld + i];
    }
}

// The same Jacobi method for n <= 16 with the work of a round split by 2 x 2
// blocks: in a round the pairs partition the indices, so lane (I, J) (I, J <
// n/2 rounded up) owns the block of rows {p_I, q_I} and columns {p_J, q_J}.
// The two-sided rotation of that block reads only the block (rows by pair I,
// then columns by pair J), and so does the column rotation of V on rows
// {2I, 2I + 1}: every lane reads, rotates and writes its own elements, and a
// round needs one barrier after the parameters and one after the update.
// The pair order, the skip test and the stopping rule are those above.
template <int NT>
__global__ __launch_bounds__(64) void eig_herm_blk_kernel(cd* __restrict__ Aall, int n_arg,
                                                          double* __restrict__ w_out,
                                                          cd* __restrict__ V_out) {
    const int n = NT > 0 ? NT : n_arg;
    constexpr int LD = 17;  // odd row stride (see above)
    __shared__ cd A[16 * LD], V[16 * LD];
    __shared__ double prm[8][4];  // c, s, e of every pair of the round
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x;
    const int I = lane >> 3, J = lane & 7;
    const int np = n + (n & 1), half = np / 2;
    const bool act = I < half && J < half;
    const cd* Ag = Aall + b * (int64_t)n * n;
    for (int i = lane; i < n * n; i += 64) {
        const int r = i / n, c = i - r * n;
        A[r * LD + c] = Ag[i];
        V[r * LD + c] = cd{r == c ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    const double eps2 = 4.9e-32;  // (2.2e-16)^2
    for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = lane; i < n * n; i += 64) {
            const int r = i / n, c = i - r * n;
            const double v = cabs2(A[r * LD + c]);
            if (r == c)
                dia += v;
            else
                off += v;
        }
        off = wave_sum(off);
        dia = wave_sum(dia);
        if (!(off > 1e-32 * dia)) break;
        const double skip_abs = eps2 * dia / n;
        int rotated = 0;
        for (int round = 0; round < np - 1; ++round) {
            if (lane < half) {
                int p, q;
                rr_pair(lane, round, np, p, q);
                double c = 1.0, s = 0.0;
                cd e = {1.0, 0.0};
                if (q < n) {
                    const double a = A[p * LD + p].x, d = A[q * LD + q].x;
                    const cd bpq = A[p * LD + q];
                    const double bb2 = cabs2(bpq);
                    if (bb2 > fmax(eps2 * fabs(a * d), skip_abs) && bb2 > 0.0) {
                        rotated = 1;
                        // (one reciprocal square root for 1/|b|, one for c: two
                        // divisions and a square root fewer on the round's critical path)
                        const double ib = rsqrt(bb2);
                        const double tau = (d - a) * (0.5 * ib);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(fma(tau, tau, 1.0)));
                        c = rsqrt(fma(t, t, 1.0));
                        s = t * c;
                        e = cd{bpq.x * ib, bpq.y * ib};
                    }
                }
                prm[lane][0] = c;
                prm[lane][1] = s;
                prm[lane][2] = e.x;
                prm[lane][3] = e.y;
            }
            __syncthreads();
            if (act) {
                int pI, qI, pJ, qJ;
                rr_pair(I, round, np, pI, qI);
                rr_pair(J, round, np, pJ, qJ);
                const double cI = prm[I][0], sI = prm[I][1], cJ = prm[J][0], sJ = prm[J][1];
                const cd eI = {prm[I][2], prm[I][3]}, eJ = {prm[J][2], prm[J][3]};
                const bool qIok = qI < n, qJok = qJ < n;
                if (sI != 0.0 || sJ != 0.0) {
                    const cd z = {0.0, 0.0};
                    cd x00 = A[pI * LD + pJ];
                    cd x01 = qJok ? A[pI * LD + qJ] : z;
                    cd x10 = qIok ? A[qI * LD + pJ] : z;
                    cd x11 = qIok && qJok ? A[qI * LD + qJ] : z;
                    if (sI != 0.0) {  // rows: A'_p = c A_p - s e A_q ; A'_q = s conj(e) A_p + c A_q
                        const cd e0 = cmul(eI, x10), e1 = cmul(eI, x11);
                        const cd f0 = cmulc(eI, x00), f1 = cmulc(eI, x01);
                        x00 = cd{cI * x00.x - sI * e0.x, cI * x00.y - sI * e0.y};
                        x01 = cd{cI * x01.x - sI * e1.x, cI * x01.y - sI * e1.y};
                        x10 = cd{sI * f0.x + cI * x10.x, sI * f0.y + cI * x10.y};
                        x11 = cd{sI * f1.x + cI * x11.x, sI * f1.y + cI * x11.y};
                    }
                    if (sJ != 0.0) {  // columns: A'_ip = c A_ip - s conj(e) A_iq ; A'_iq = s e A_ip + c A_iq
                        const cd e0 = cmulc(eJ, x01), e1 = cmulc(eJ, x11);
                        const cd f0 = cmul(eJ, x00), f1 = cmul(eJ, x10);
                        x00 = cd{cJ * x00.x - sJ * e0.x, cJ * x00.y - sJ * e0.y};
                        x10 = cd{cJ * x10.x - sJ * e1.x, cJ * x10.y - sJ * e1.y};
                        x01 = cd{sJ * f0.x + cJ * x01.x, sJ * f0.y + cJ * x01.y};
                        x11 = cd{sJ * f1.x + cJ * x11.x, sJ * f1.y + cJ * x11.y};
                    }
                    if (I == J && sI != 0.0) {  // the rotated pair: exact zero off the diagonal
                        x01 = z;
                        x10 = z;
                        x00.y = 0.0;
                        x11.y = 0.0;
                    }
                    A[pI * LD + pJ] = x00;
                    if (qJok) A[pI * LD + qJ] = x01;
                    if (qIok) A[qI * LD + pJ] = x10;
                    if (qIok && qJok) A[qI * LD + qJ] = x11;
                }
                if (sJ != 0.0) {  // V columns p_J, q_J on rows 2I, 2I + 1
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int r = 2 * I + h;
                        if (r < n) {
                            const cd vp = V[r * LD + pJ];
                            const cd vq = qJok ? V[r * LD + qJ] : cd{0.0, 0.0};
                            const cd eq = cmulc(eJ, vq), ep = cmul(eJ, vp);
                            V[r * LD + pJ] = cd{cJ * vp.x - sJ * eq.x, cJ * vp.y - sJ * eq.y};
                            if (qJok) V[r * LD + qJ] = cd{sJ * ep.x + cJ * vq.x, sJ * ep.y + cJ * vq.y};
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (!__any(rotated)) break;  // a sweep with no rotation leaves A unchanged
    }
    // ascending order, ties by index
    for (int i = lane; i < n; i += 64) {
        const double wi = A[i * LD + i].x;
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double wj = A[j * LD + j].x;
            rank += (wj < wi) || (wj == wi && j < i);
        }
        w_out[b * n + rank] = wi;
        cd* Vg = V_out + b * (int64_t)n * n;
        for (int r = 0; r < n; ++r) Vg[r * n + rank] = V[r * LD + i];
    }
}

hipError_t launch_eig_herm(cd* A, int n, int64_t batch, double* w, cd* V, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    const int h = n / 2 + 1;
    const size_t shm = (size_t)2 * n * (n + 1) * sizeof(cd) + 2 * h * sizeof(double) +
                       h * sizeof(cd) + 2 * h * sizeof(int);
    for (int64_t b0 = 0; b0 < batch; b0 += 2000000000LL) {
        const int64_t nb = batch - b0 < 2000000000LL ? batch - b0 : 2000000000LL;
        cd* Ab = A + b0 * n * n;
        double* wb = w + b0 * n;
        cd* Vb = V + b0 * n * n;
        switch (n) {
#define PHX_EIG(NV)                                                                             \
    case NV:                                                                                    \
        hipLaunchKernelGGL(eig_herm_kernel<NV>, dim3((unsigned)nb), dim3(64), shm, s, Ab, n, wb, \
                           Vb);                                                                 \
        break;
#define PHX_EIGB(NV)                                                                            \
    case NV:                                                                                    \
        hipLaunchKernelGGL(eig_herm_blk_kernel<NV>, dim3((unsigned)nb), dim3(64), 0, s, Ab, n,  \
                           wb, Vb);                                                             \
        break;
            PHX_EIGB(3) PHX_EIGB(4) PHX_EIGB(5) PHX_EIGB(6) PHX_EIGB(7) PHX_EIGB(8) PHX_EIGB(9)
            PHX_EIGB(10) PHX_EIGB(12) PHX_EIGB(14) PHX_EIGB(15) PHX_EIGB(16)
            PHX_EIG(18) PHX_EIG(20) PHX_EIG(21) PHX_EIG(24) PHX_EIG(27) PHX_EIG(30)
            case 1: case 2: case 11: case 13:
                hipLaunchKernelGGL(eig_herm_blk_kernel<0>, dim3((unsigned)nb), dim3(64), 0, s, Ab,
                                   n, wb, Vb);
                break;
#undef PHX_EIG
#undef PHX_EIGB
            default:
                hipLaunchKernelGGL(eig_herm_kernel<0>, dim3((unsigned)nb), dim3(64), shm, s, Ab, n,
                                   wb, Vb);
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phonon post-processing and occupations
// ---------------------------------------------------------------------------
__global__ void phonon_post_kernel(const double* lam, const cd* z, const double* mass, int nat,
                                   int64_t nq, double omega_min, double kT, double c_om,
                                   double c_ph, double* omega, cd* e, double* nb) {
    const int nm = 3 * nat;
    const int64_t total = nq * nm;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = t / nm;
        const int nu = (int)(t % nm);
        const double l = lam[t];
        const double w = c_om * sqrt(l > 0.0 ? l : 0.0);
        const bool act = w >= omega_min && w > 0.0;
        if (omega) omega[t] = w;
        if (nb) nb[t] = (act && kT > 0.0) ? 1.0 / expm1(w / kT) : 0.0;
        if (e) {
            // E[q, nu, sa] = z[q][sa][nu] l_{sa,nu}: one mode's column contiguous
            for (int sa = 0; sa < nm; ++sa) {
                const int64_t o = (q * nm + sa) * nm + nu;
                const int64_t oe = (q * nm + nu) * nm + sa;
                if (act) {
                    const double ls = sqrt(c_ph / (2.0 * mass[sa / 3] * w));
                    e[oe] = cd{z[o].x * ls, z[o].y * ls};
                } else {
                    e[oe] = cd{0.0, 0.0};
                }
            }
        }
    }
}

hipError_t launch_phonon_post(const double* lam, const cd* z, const double* mass, int nat,
                              int64_t nq, double omega_min, double kT, double* omega, cd* e,
                              double* nb, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(phonon_post_kernel, dim3(grid_for(nq * 3 * nat, 256)), dim3(256), 0, s, lam,
                       z, mass, nat, nq, omega_min, kT, c_omega(), kCPh, omega, e, nb);
    return hipGetLastError();
}

__global__ void fermi_kernel(const double* eps, int64_t n, double mu, double kT, double* f) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const double x = (eps[t] - mu) / kT;
        if (x > 0.0) {
            const double ex = exp(-x);
            f[t] = ex / (1.0 + ex);
        } else {
            f[t] = 1.0 / (1.0 + exp(x));
        }
    }
}

hipError_t launch_fermi(const double* eps, int64_t n, double mu, double kT, double* f,
                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fermi_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, eps, n, mu, kT, f);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Window, ordered compaction, band extrema
// ---------------------------------------------------------------------------
__global__ void window_kernel(const double* eps, int64_t nk, int nW, double lo, double hi,
                              uint8_t* mask, int32_t* flag) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nk;
         k += (int64_t)gridDim.x * blockDim.x) {
        int any = 0;
        for (int b = 0; b < nW; ++b) {
            const double e = eps[k * nW + b];
            const int in = (e > lo) && (e < hi);
            if (mask) mask[k * nW + b] = (uint8_t)in;
            any |= in;
        }
        if (flag) flag[k] = any;
    }
}

hipError_t launch_window(const double* eps, int64_t nk, int nW, double lo, double hi,
                         uint8_t* mask, int32_t* flag, hipStream_t s) {
    if (nk <= 0) return hipSuccess;
    hipLaunchKernelGGL(window_kernel, dim3(grid_for(nk, 256)), dim3(256), 0, s, eps, nk, nW, lo,
                       hi, mask, flag);
    return hipGetLastError();
}

// One work-group of 1024 threads scans the flags chunk by chunk in order.
__global__ __launch_bounds__(1024) void compact_kernel(const int32_t* flag, int64_t n, int32_t* out,
                                                        int32_t* count) {
    __shared__ int32_t wsum[16];
    __shared__ int32_t base_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) base_sh = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < n; c0 += 1024) {
        const int64_t i = c0 + tid;
        const int f = (i < n && flag[i] != 0) ? 1 : 0;
        // inclusive scan within the wave
        int v = f;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(v, o, 64);
            if (lane >= o) v += u;
        }
        if (lane == 63) wsum[wave] = v;
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        const int base = base_sh;
        if (f) out[base + before + v - 1] = (int32_t)i;
        __syncthreads();
        if (tid == 1023) base_sh = base + before + v;
        __syncthreads();
    }
    if (tid == 0) *count = base_sh;
}

hipError_t launch_compact(const int32_t* flag, int64_t n, int32_t* out, int32_t* count,
                          hipStream_t s) {
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(1024), 0, s, flag, n, out, count);
    return hipGetLastError();
}

// min and max are exact in any order; the loads of a thread are unrolled so that
// eight are in flight at once
__global__ __launch_bounds__(1024) void extrema_kernel(const double* eps, int64_t nk, int nW,
                                                       const double* omega, int64_t nq, int nm,
                                                       double* bmin, double* bmax, double* wmax) {
    __shared__ double s1[1024], s2[1024];
    const int b = blockIdx.x;  // b < nW: band b; b == nW: phonon maximum
    double lo = 1e300, hi = -1e300;
    if (b < nW) {
#pragma unroll 8
        for (int64_t k = threadIdx.x; k < nk; k += 1024) {
            const double e = eps[k * nW + b];
            lo = fmin(lo, e);
            hi = fmax(hi, e);
        }
    } else {
#pragma unroll 8
        for (int64_t t = threadIdx.x; t < nq * nm; t += 1024) hi = fmax(hi, omega[t]);
    }
    s1[threadIdx.x] = lo;
    s2[threadIdx.x] = hi;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s1[threadIdx.x] = fmin(s1[threadIdx.x], s1[threadIdx.x + o]);
            s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (b < nW) {
            bmin[b] = s1[0];
            bmax[b] = s2[0];
        } else {
            *wmax = s2[0];
        }
    }
}

hipError_t launch_band_extrema(const double* eps, int64_t nk, int nW, const double* omega,
                               int64_t nq, int nm, double* bmin, double* bmax, double* wmax,
                               hipStream_t s) {
    hipLaunchKernelGGL(extrema_kernel, dim3(nW + 1), dim3(1024), 0, s, eps, nk, nW, omega, nq, nm,
                       bmin, bmax, wmax);
    return hipGetLastError();
}

__global__ void kq_kernel(const double* k, int64_t nk, const double* q, int64_t nq, double* kq) {
    const int64_t total = nk * nq;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / nq, j = t % nq;
        for (int d = 0; d < 3; ++d) kq[3 * t + d] = k[3 * i + d] + q[3 * j + d];
    }
}

hipError_t launch_kq_points(const double* k, int64_t nk, const double* q, int64_t nq,
                            double* kq, hipStream_t s) {
    if (nk * nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(kq_kernel, dim3(grid_for(nk * nq, 256)), dim3(256), 0, s, k, nk, q, nq, kq);
    return hipGetLastError();
}

// Bands at k + q for k and q on one mesh: the mesh's bands gathered per pair.
// Pair (i, j) of k index k_idx[i] and q index j takes mesh point
// ((k0 + q0) mod N0, (k1 + q1) mod N1, (k2 + q2) mod N2); one thread per (pair, entry).
__global__ void gather_kq_bands_kernel(const double* __restrict__ eps, const cd* __restrict__ U,
                                       int nW, Mesh m, const int32_t* __restrict__ k_idx,
                                       int64_t nk, int64_t nq, double* __restrict__ eps_kq,
                                       cd* __restrict__ Ukq) {
    const int64_t per = (int64_t)nW + (int64_t)nW * nW;
    const int64_t total = nk * nq * per;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pair = t / per;
        const int64_t e = t - pair * per;
        const int64_t i = pair / nq, j = pair - i * nq;
        int k0, k1, k2, q0, q1, q2;
        mesh_triple(k_idx[i], m, k0, k1, k2);
        mesh_triple(j, m, q0, q1, q2);
        const int64_t kq = mesh_linear((k0 + q0) % m.n0, (k1 + q1) % m.n1, (k2 + q2) % m.n2, m);
        if (e < nW)
            eps_kq[pair * nW + e] = eps[kq * nW + e];
        else
            Ukq[pair * nW * nW + (e - nW)] = U[kq * nW * nW + (e - nW)];
    }
}

hipError_t launch_gather_kq_bands(const double* eps, const cd* U, int nW, Mesh m,
                                  const int32_t* k_idx, int64_t nk, int64_t nq, double* eps_kq,
                                  cd* Ukq, hipStream_t s) {
    if (nk * nq <= 0) return hipSuccess;
    const int64_t total = nk * nq * ((int64_t)nW + (int64_t)nW * nW);
    hipLaunchKernelGGL(gather_kq_bands_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, eps, U,
                       nW, m, k_idx, nk, nq, eps_kq, Ukq);
    return hipGetLastError();
}

// Fill with zeros by a kernel (safe under stream capture).
__global__ void zero_kernel(uint32_t* p, int64_t n, uint8_t* tail, int ntail) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0u;
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    // buffers come from the workspace or the caller and are at least 4-byte aligned
    const int64_t n = (int64_t)(bytes / 4);
    const int ntail = (int)(bytes % 4);
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n > 0 ? n : 1, 256)), dim3(256), 0, s,
                       (uint32_t*)p, n, (uint8_t*)p + 4 * n, ntail);
    return hipGetLastError();
}

}  // namespace phx
