// Kernels beyond the plain rate path (see ext.hpp): the polar long-range
// factor, group velocities, the phonon-linewidth reduction, Philox streams,
// network initialisation, training-set selection, row gathers, the
// finiteness scan and the 3-phonon coupling contractions.
#include <algorithm>

#include "ext.hpp"

namespace phx {

static inline unsigned grid_n(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65535 * 16) g = 65535 * 16;  // grid-stride loops take the rest
    return (unsigned)g;
}

// ---------------------------------------------------------------------------
// Polar long-range factor (Electron Properties, long-range coupling)
// ---------------------------------------------------------------------------
__global__ void polar_factor_kernel(const double* frac, Mesh m, int64_t np, const cd* E, int nm,
                                    PolarDev pd, double pref, cd* L) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np;
         p += (int64_t)gridDim.x * blockDim.x) {
        double q[3];
        if (frac) {
            q[0] = frac[3 * p];
            q[1] = frac[3 * p + 1];
            q[2] = frac[3 * p + 2];
        } else {
            int i0, i1, i2;
            mesh_triple(p, m, i0, i1, i2);
            q[0] = (double)i0 / m.n0;
            q[1] = (double)i1 / m.n1;
            q[2] = (double)i2 / m.n2;
        }
        double D[30];
        for (int i = 0; i < 3 * pd.nat; ++i) D[i] = 0.0;
        const int gm = pd.g_max;
        for (int g0 = -gm; g0 <= gm; ++g0)
            for (int g1 = -gm; g1 <= gm; ++g1)
                for (int g2 = -gm; g2 <= gm; ++g2) {
                    const double K0 = 2.0 * kPi * (q[0] + g0), K1 = 2.0 * kPi * (q[1] + g1),
                                 K2 = 2.0 * kPi * (q[2] + g2);
                    if (sqrt(K0 * K0 + K1 * K1 + K2 * K2) <= 1e-12) continue;  // q + G = 0
                    const double* e = pd.eps;
                    const double den = K0 * (e[0] * K0 + e[1] * K1 + e[2] * K2) +
                                       K1 * (e[3] * K0 + e[4] * K1 + e[5] * K2) +
                                       K2 * (e[6] * K0 + e[7] * K1 + e[8] * K2);
                    const double w = exp(-den / (4.0 * pd.alpha)) / den;
                    for (int s = 0; s < pd.nat; ++s) {
                        const double* Z = pd.born + 9 * s;
                        for (int b = 0; b < 3; ++b)
                            D[3 * s + b] += w * (K0 * Z[b] + K1 * Z[3 + b] + K2 * Z[6 + b]);
                    }
                }
        const cd* Ep = E + p * nm * nm;
        for (int nu = 0; nu < nm; ++nu) {
            cd acc = {0.0, 0.0};
            for (int sa = 0; sa < nm; ++sa) {
                const cd e = Ep[nu * nm + sa];
                acc.x += D[sa] * e.x;
                acc.y += D[sa] * e.y;
            }
            L[p * nm + nu] = cd{pref * acc.x, pref * acc.y};
        }
    }
}

hipError_t launch_polar_factor(const double* frac, Mesh m, int64_t np, const cd* E, int nm,
                               const PolarDev& pd, cd* L, hipStream_t s) {
    if (np <= 0) return hipSuccess;
    if (pd.nat > 10 || nm != 3 * pd.nat) return hipErrorInvalidValue;
    // 4 pi (e^2 / (4 pi eps0)) in eV A^2 for V = 1 A^3 (CODATA 2018: e / (4 pi eps0 A))
    const double e2 = 1.602176634e-19 / (4.0 * kPi * 8.8541878128e-12 * 1.0e-10);
    hipLaunchKernelGGL(polar_factor_kernel, dim3(grid_n(np, 128)), dim3(128), 0, s, frac, m, np, E,
                       nm, pd, 4.0 * kPi * e2, L);
    return hipGetLastError();
}

__global__ void polar_add_g_kernel(cd* g, int64_t nq, const cd* Uk, const cd* Ukq, const cd* L,
                                   int nW, int nm) {
    const int64_t total = nq * nW * nW;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int mm = (int)(t % nW);
        const int n = (int)((t / nW) % nW);
        const int64_t q = t / ((int64_t)nW * nW);
        const cd* Uq = Ukq + q * nW * nW;
        cd o = {0.0, 0.0};
        for (int a = 0; a < nW; ++a) o = cfmac(Uk[a * nW + n], Uq[a * nW + mm], o);
        cd* gq = g + q * nm * nW * nW + n * nW + mm;
        for (int nu = 0; nu < nm; ++nu) {
            const cd l = L[q * nm + nu];
            // i L O
            const cd lo = cmul(l, o);
            cd v = gq[(int64_t)nu * nW * nW];
            v.x -= lo.y;
            v.y += lo.x;
            gq[(int64_t)nu * nW * nW] = v;
        }
    }
}

hipError_t launch_polar_add_g(cd* g, int64_t nq, const cd* Uk, const cd* Ukq, const cd* L,
                              int nW, int nm, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(polar_add_g_kernel, dim3(grid_n(nq * nW * nW, 256)), dim3(256), 0, s, g, nq,
                       Uk, Ukq, L, nW, nm);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Group velocities (Electron Properties, Velocity)
// ---------------------------------------------------------------------------
__global__ void velocity_phases_kernel(const cd* P, int64_t np, const int32_t* R, int nR, cd* Pv) {
    const int64_t total = np * 3 * nR;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(t % nR);
        const int a = (int)((t / nR) % 3);
        const int64_t p = t / (3 * (int64_t)nR);
        const double ra = (double)R[3 * r + a];
        const cd ph = P[p * nR + r];
        Pv[t] = cd{-ra * ph.y, ra * ph.x};  // i R_a e^{i 2 pi k.R}
    }
}

hipError_t launch_velocity_phases(const cd* P, int64_t np, const int32_t* R, int nR, cd* Pv,
                                  hipStream_t s) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(velocity_phases_kernel, dim3(grid_n(np * 3 * nR, 256)), dim3(256), 0, s, P,
                       np, R, nR, Pv);
    return hipGetLastError();
}

// Eigenvalues (ascending) of a Hermitian n x n matrix (n <= 8) by cyclic Jacobi:
// each rotation first turns A_pq real with a phase on index q, then zeroes it
// with a real plane rotation.
__device__ void herm_eigvals_small(cd (*A)[8], int n, double* w) {
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int p = 0; p < n; ++p) {
            dia += A[p][p].x * A[p][p].x;
            for (int q = p + 1; q < n; ++q) off += cabs2(A[p][q]);
        }
        if (off <= 1e-32 * (dia + 1e-300)) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double r = sqrt(cabs2(A[p][q]));
                if (r == 0.0) continue;
                const cd ph = {A[p][q].x / r, A[p][q].y / r};  // e^{i phi}
                for (int k = 0; k < n; ++k) {
                    A[k][q] = cmulc(ph, A[k][q]);                 // column q times e^{-i phi}
                    A[q][k] = cmul(ph, A[q][k]);                  // row q times e^{i phi}
                }
                const double th = (A[q][q].x - A[p][p].x) / (2.0 * r);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {
                    const cd akp = A[k][p], akq = A[k][q];
                    A[k][p] = cd{c * akp.x - sn * akq.x, c * akp.y - sn * akq.y};
                    A[k][q] = cd{sn * akp.x + c * akq.x, sn * akp.y + c * akq.y};
                }
                for (int k = 0; k < n; ++k) {
                    const cd apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cd{c * apk.x - sn * aqk.x, c * apk.y - sn * aqk.y};
                    A[q][k] = cd{sn * apk.x + c * aqk.x, sn * apk.y + c * aqk.y};
                }
            }
    }
    for (int i = 0; i < n; ++i) w[i] = A[i][i].x;
    for (int i = 1; i < n; ++i) {  // insertion sort, ascending
        const double x = w[i];
        int j = i - 1;
        while (j >= 0 && w[j] > x) {
            w[j + 1] = w[j];
            --j;
        }
        w[j + 1] = x;
    }
}

__global__ void group_velocities_kernel(const cd* dH, const cd* U, int utr, const double* eps,
                                        int64_t np, int nW, double tol, double* v, int32_t* bad) {
    const int64_t total = np * 3;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(t % 3);
        const int64_t p = t / 3;
        const cd* H = dH + t * nW * nW;  // [p, a] block
        const cd* Up = U + p * nW * nW;
        const double* e = eps + p * nW;
        // U[orbital, band]
        auto u = [&](int orb, int band) { return utr ? Up[band * nW + orb] : Up[orb * nW + band]; };
        // V_nm = sum_b conj(U[b, n]) sum_c dH[b, c] U[c, m]
        auto vel = [&](int n, int mm) {
            cd acc = {0.0, 0.0};
            for (int b = 0; b < nW; ++b) {
                cd hu = {0.0, 0.0};
                for (int c = 0; c < nW; ++c) hu = cfma(H[b * nW + c], u(c, mm), hu);
                acc = cfmac(u(b, n), hu, acc);
            }
            return acc;
        };
        int b0 = 0;
        while (b0 < nW) {
            int b1 = b0 + 1;
            while (b1 < nW && fabs(e[b1] - e[b1 - 1]) < tol) ++b1;
            const int g = b1 - b0;
            if (g == 1) {
                v[(p * nW + b0) * 3 + a] = vel(b0, b0).x;
            } else if (g <= 8) {
                cd A[8][8];
                for (int i = 0; i < g; ++i)
                    for (int j = 0; j < g; ++j) A[i][j] = vel(b0 + i, b0 + j);
                double w[8];
                herm_eigvals_small(A, g, w);
                for (int i = 0; i < g; ++i) v[(p * nW + b0 + i) * 3 + a] = w[i];
            } else {
                for (int i = 0; i < g; ++i) v[(p * nW + b0 + i) * 3 + a] = 0.0;
                *bad = 1;
            }
            b0 = b1;
        }
    }
}

hipError_t launch_group_velocities(const cd* dH, const cd* U, bool u_transposed,
                                   const double* eps, int64_t np, int nW, double tol, double* v,
                                   int32_t* bad, hipStream_t s) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(group_velocities_kernel, dim3(grid_n(np * 3, 64)), dim3(64), 0, s, dH, U,
                       u_transposed ? 1 : 0, eps, np, nW, tol, v, bad);
    return hipGetLastError();
}

__global__ __launch_bounds__(1024) void velocity_max_kernel(const double* v, int64_t n3,
                                                            double* vmax) {
    __shared__ double sm[3][1024];
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int64_t i = threadIdx.x; i < n3; i += 1024) {
        m0 = fmax(m0, fabs(v[3 * i]));
        m1 = fmax(m1, fabs(v[3 * i + 1]));
        m2 = fmax(m2, fabs(v[3 * i + 2]));
    }
    sm[0][threadIdx.x] = m0;
    sm[1][threadIdx.x] = m1;
    sm[2][threadIdx.x] = m2;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int d = 0; d < 3; ++d) sm[d][threadIdx.x] = fmax(sm[d][threadIdx.x], sm[d][threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x < 3) vmax[threadIdx.x] = sm[threadIdx.x][0];
}

hipError_t launch_velocity_max(const double* v, int64_t np, int nW, double* vmax, hipStream_t s) {
    hipLaunchKernelGGL(velocity_max_kernel, dim3(1), dim3(1024), 0, s, v, np * nW, vmax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Phonon linewidth (Transport Methods, phonon BTE): sums over states in order
// ---------------------------------------------------------------------------
__global__ void lw_reduce_lines_kernel(const double* lw, const uint32_t* line_bands,
                                       const uint32_t* live, int nst, int NL, int N0, int nm,
                                       double* acc) {
    const int64_t per = (int64_t)N0 * nm;
    const int64_t total = (int64_t)NL * per;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int line = (int)(t / per);
        const int64_t j = t - line * per;  // q0 nm + nu
        double s = 0.0;
        const int q0 = (int)(j / nm), nu = (int)(j - (int64_t)q0 * nm);
        // a (state, line) pair's partials exist at its live points only
        for (int st = 0; st < nst; ++st)
            if (line_bands[(int64_t)st * NL + line] && live[((int64_t)st * NL + line) * N0 + q0])
                s += lw[((int64_t)st * NL + line) * per + j];
        acc[((int64_t)q0 * NL + line) * nm + nu] += s;
    }
}

hipError_t launch_lw_reduce_lines(const double* lw, const uint32_t* line_bands,
                                  const uint32_t* live, int nst, int NL, int N0, int nm,
                                  double* acc, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    hipLaunchKernelGGL(lw_reduce_lines_kernel, dim3(grid_n((int64_t)NL * N0 * nm, 256)), dim3(256),
                       0, s, lw, line_bands, live, nst, NL, N0, nm, acc);
    return hipGetLastError();
}

__global__ void lw_reduce_dense_kernel(const double* lw, int nst, int64_t N, int nm, double* acc) {
    const int64_t per = N * nm;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < per;
         t += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int st = 0; st < nst; ++st) s += lw[(int64_t)st * per + t];
        acc[t] += s;
    }
}

hipError_t launch_lw_reduce_dense(const double* lw, int nst, int64_t N, int nm, double* acc,
                                  hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    hipLaunchKernelGGL(lw_reduce_dense_kernel, dim3(grid_n(N * nm, 256)), dim3(256), 0, s, lw, nst,
                       N, nm, acc);
    return hipGetLastError();
}

__global__ void lw_finish_kernel(const double* acc, const double* omega, const double* nb,
                                 int64_t n, double omega_min, double scale, double* P) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const double w = omega[t];
        const double b = nb[t];
        P[t] = (w >= omega_min && w > 0.0) ? scale * b * (b + 1.0) * w * acc[t] : 0.0;
    }
}

hipError_t launch_lw_finish(const double* acc, const double* omega, const double* nb, int64_t n,
                            double omega_min, double scale, double* P, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(lw_finish_kernel, dim3(grid_n(n, 256)), dim3(256), 0, s, acc, omega, nb, n,
                       omega_min, scale, P);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Philox-4x64-10 (Salmon et al., SC'11): word 0 of the block with counter
// (c, 0, 0, 0) and key (seed, 0)
// ---------------------------------------------------------------------------
__device__ inline uint64_t philox_w0(uint64_t c, uint64_t seed) {
    uint64_t x0 = c, x1 = 0, x2 = 0, x3 = 0, k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = x0 * 0xD2E7470EE14C6C93ull, hi0 = __umul64hi(x0, 0xD2E7470EE14C6C93ull);
        const uint64_t lo1 = x2 * 0xCA5A826395121157ull, hi1 = __umul64hi(x2, 0xCA5A826395121157ull);
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    return x0;
}
__device__ inline double philox_uniform(uint64_t c, uint64_t seed) {
    return (double)(philox_w0(c, seed) >> 11) * 0x1.0p-53;
}

__global__ void philox_uniform_kernel(uint64_t seed, uint64_t offset, int64_t n, double* out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        out[t] = philox_uniform(offset + (uint64_t)t, seed);
}

__global__ void philox_randint_kernel(uint64_t seed, uint64_t offset, int64_t n, double hi,
                                      int32_t* out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        out[t] = (int32_t)floor(philox_uniform(offset + (uint64_t)t, seed) * hi);
}

hipError_t launch_philox_uniform(uint64_t seed, uint64_t offset, int64_t n, double* out,
                                 hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_uniform_kernel, dim3(grid_n(n, 256)), dim3(256), 0, s, seed, offset, n,
                       out);
    return hipGetLastError();
}

hipError_t launch_philox_randint(uint64_t seed, uint64_t offset, int64_t n, int64_t hi,
                                 int32_t* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_randint_kernel, dim3(grid_n(n, 256)), dim3(256), 0, s, seed, offset, n,
                       (double)hi, out);
    return hipGetLastError();
}

__global__ void uniform_fill_kernel(void* params, int f64, uint64_t seed, int64_t off,
                                    int64_t count, double div) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = off + t;
        const double w = (2.0 * philox_uniform((uint64_t)j, seed) - 1.0) / div;
        if (f64)
            static_cast<double*>(params)[j] = w;
        else
            static_cast<float*>(params)[j] = (float)w;
    }
}

hipError_t launch_uniform_fill(void* params, bool f64, uint64_t seed, int64_t off, int64_t count,
                               double div, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(uniform_fill_kernel, dim3(grid_n(count, 256)), dim3(256), 0, s, params,
                       f64 ? 1 : 0, seed, off, count, div);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Training set of the learned proposal
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ts_state_max_kernel(const double* D, int64_t per,
                                                           double* dmax) {
    __shared__ double sm[256];
    const double* d = D + (int64_t)blockIdx.x * per;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < per; i += 256) m = fmax(m, d[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dmax[blockIdx.x] = sm[0];
}

hipError_t launch_ts_state_max(const double* D, int64_t ns, int64_t per, double* dmax,
                               hipStream_t s) {
    if (ns <= 0) return hipSuccess;
    if (ns > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(ts_state_max_kernel, dim3((unsigned)ns), dim3(256), 0, s, D, per, dmax);
    return hipGetLastError();
}

// A fixed grid of kTsBlocks work-groups: each thread's entries and every sum's
// order are the same on every call.
__global__ __launch_bounds__(256) void ts_stats_kernel(const double* T, const double* D,
                                                       const double* dmax, int64_t ns, int64_t per,
                                                       double thr, double* partial) {
    __shared__ double sc[256], sr[256];
    const int64_t total = ns * per;
    double cnt = 0.0, sum = 0.0;
    for (int64_t t = blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)kTsBlocks * 256) {
        const double d = D[t];
        if (d > thr * dmax[t / per]) {
            cnt += 1.0;
            sum += T[t] / d;
        }
    }
    sc[threadIdx.x] = cnt;
    sr[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sc[threadIdx.x] += sc[threadIdx.x + o];
            sr[threadIdx.x] += sr[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sc[0];
        partial[2 * blockIdx.x + 1] = sr[0];
    }
}

__global__ void ts_stats_final_kernel(const double* partial, double* stats) {
    double c = 0.0, r = 0.0;
    for (int b = 0; b < kTsBlocks; ++b) {
        c += partial[2 * b];
        r += partial[2 * b + 1];
    }
    stats[0] = c;
    stats[1] = r;
}

hipError_t launch_ts_stats(const double* T, const double* D, const double* dmax, int64_t ns,
                           int64_t per, double thr, double* partial, double* stats,
                           hipStream_t s) {
    hipLaunchKernelGGL(ts_stats_kernel, dim3(kTsBlocks), dim3(256), 0, s, T, D, dmax, ns, per, thr,
                       partial);
    hipLaunchKernelGGL(ts_stats_final_kernel, dim3(1), dim3(1), 0, s, partial, stats);
    return hipGetLastError();
}

__device__ inline bool ts_keep(const double* D, const double* dmax, int64_t t, int64_t per,
                               double thr, uint64_t seed, double p_keep) {
    return D[t] > thr * dmax[t / per] && philox_uniform((uint64_t)t, seed) < p_keep;
}

// one work-group per chunk of kTsChunk entries: number of kept entries
__global__ __launch_bounds__(256) void ts_count_kernel(const double* D, const double* dmax,
                                                       int64_t total, int64_t per, double thr,
                                                       uint64_t seed, double p_keep,
                                                       int32_t* counts) {
    __shared__ int sm[4];
    const int64_t c0 = (int64_t)blockIdx.x * kTsChunk;
    int n = 0;
    for (int i = threadIdx.x; i < kTsChunk; i += 256) {
        const int64_t t = c0 + i;
        if (t < total && ts_keep(D, dmax, t, per, thr, seed, p_keep)) ++n;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = sm[0] + sm[1] + sm[2] + sm[3];
}

hipError_t launch_ts_count(const double* D, const double* dmax, int64_t ns, int64_t per, double thr,
                           uint64_t seed, double p_keep, int32_t* counts, hipStream_t s) {
    const int64_t total = ns * per;
    const int64_t nch = (total + kTsChunk - 1) / kTsChunk;
    if (nch <= 0) return hipSuccess;
    if (nch > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(ts_count_kernel, dim3((unsigned)nch), dim3(256), 0, s, D, dmax, total, per,
                       thr, seed, p_keep, counts);
    return hipGetLastError();
}

// One work-group of 1024 threads: in-place exclusive scan, chunk by chunk.
__global__ __launch_bounds__(1024) void exclusive_scan_kernel(int32_t* x, int64_t n,
                                                              int64_t* total) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t base_sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) base_sh = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < n; c0 += 1024) {
        const int64_t i = c0 + tid;
        const int64_t f = i < n ? x[i] : 0;
        int64_t v = f;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t u = __shfl_up(v, o, 64);
            if (lane >= o) v += u;
        }
        if (lane == 63) wsum[wave] = v;
        __syncthreads();
        int64_t before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        const int64_t base = base_sh;
        if (i < n) x[i] = (int32_t)(base + before + v - f);
        __syncthreads();
        if (tid == 1023) base_sh = base + before + v;
        __syncthreads();
    }
    if (tid == 0) *total = base_sh;
}

hipError_t launch_exclusive_scan(int32_t* counts, int64_t n, int64_t* total, hipStream_t s) {
    hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(1024), 0, s, counts, n, total);
    return hipGetLastError();
}

// Kept entries of a chunk written in flat-index order at the chunk's offset.
__global__ __launch_bounds__(256) void ts_write_kernel(const double* T, const double* D,
                                                       const double* dmax, int64_t total,
                                                       int64_t per, int nm, int64_t nq, double thr,
                                                       uint64_t seed, double p_keep, double c,
                                                       const int32_t* offsets, int64_t cap,
                                                       int32_t* o_state, int32_t* o_q,
                                                       int32_t* o_nu, float* o_y) {
    __shared__ int wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kTsChunk;
    int64_t base = offsets[blockIdx.x];
    for (int i0 = 0; i0 < kTsChunk; i0 += 256) {
        const int64_t t = c0 + i0 + tid;
        const bool keep = t < total && ts_keep(D, dmax, t, per, thr, seed, p_keep);
        const uint64_t bal = __ballot(keep);
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        const int64_t pos = base + before + __popcll(bal & ((1ull << lane) - 1ull));
        if (keep && pos < cap) {
            const int64_t st = t / per;
            const int64_t r = t - st * per;
            const int64_t q = r / nm;
            o_state[pos] = (int32_t)st;
            o_q[pos] = (int32_t)q;
            o_nu[pos] = (int32_t)(r - q * nm);
            o_y[pos] = (float)log(T[t] / D[t] + c);
        }
        base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    (void)nq;
}

hipError_t launch_ts_write(const double* T, const double* D, const double* dmax, int64_t ns,
                           int64_t per, int nm, int64_t nq, double thr, uint64_t seed,
                           double p_keep, double c, const int32_t* offsets, int64_t cap,
                           int32_t* o_state, int32_t* o_q, int32_t* o_nu, float* o_y,
                           hipStream_t s) {
    const int64_t total = ns * per;
    const int64_t nch = (total + kTsChunk - 1) / kTsChunk;
    if (nch <= 0) return hipSuccess;
    hipLaunchKernelGGL(ts_write_kernel, dim3((unsigned)nch), dim3(256), 0, s, T, D, dmax, total, per,
                       nm, nq, thr, seed, p_keep, c, offsets, cap, o_state, o_q, o_nu, o_y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row gather, finiteness scan
// ---------------------------------------------------------------------------
__global__ void gather_rows32_kernel(const uint32_t* src, int64_t words, const int32_t* idx,
                                     int64_t n, uint32_t* dst) {
    const int64_t total = n * words;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / words, w = t - i * words;
        dst[t] = src[(int64_t)idx[i] * words + w];
    }
}

hipError_t launch_gather_rows32(const uint32_t* src, int64_t words, const int32_t* idx, int64_t n,
                                uint32_t* dst, hipStream_t s) {
    if (n <= 0 || words <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows32_kernel, dim3(grid_n(n * words, 256)), dim3(256), 0, s, src,
                       words, idx, n, dst);
    return hipGetLastError();
}

__global__ void nonfinite_kernel(const double* x, int64_t n, int32_t* flag) {
    int bad = 0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[t]);
    if (__ballot(bad) && (threadIdx.x & 63) == 0) *flag = 1;  // vector store of a constant
}

hipError_t launch_nonfinite(const double* x, int64_t n, int32_t* flag, hipStream_t s) {
    if (n <= 0 || !x) return hipSuccess;
    hipLaunchKernelGGL(nonfinite_kernel, dim3(std::min<int64_t>(grid_n(n, 256), 4096)), dim3(256),
                       0, s, x, n, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3-phonon coupling (Phonon Properties; Kokkos section, generic contraction)
// ---------------------------------------------------------------------------
__global__ void real_to_complex_kernel(const double* x, int64_t n, cd* out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        out[t] = cd{x[t], 0.0};
}

hipError_t launch_real_to_complex(const double* x, int64_t n, cd* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(real_to_complex_kernel, dim3(grid_n(n, 256)), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
}

__global__ void neg_pair_sum_kernel(const double* q, int64_t nq, const double* qp, int64_t nqp,
                                    double* out) {
    const int64_t total = nq * nqp;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / nqp, j = t - i * nqp;
        for (int d = 0; d < 3; ++d) out[3 * t + d] = -(q[3 * i + d] + qp[3 * j + d]);
    }
}

hipError_t launch_neg_pair_sum(const double* q, int64_t nq, const double* qp, int64_t nqp,
                               double* out, hipStream_t s) {
    if (nq * nqp <= 0) return hipSuccess;
    hipLaunchKernelGGL(neg_pair_sum_kernel, dim3(grid_n(nq * nqp, 256)), dim3(256), 0, s, q, nq, qp,
                       nqp, out);
    return hipGetLastError();
}

__global__ void v3_fold_kernel(const cd* S, int64_t nq, int nr, int nm, const cd* E1, cd* T) {
    const int64_t nbc = (int64_t)nm * nm;
    const int64_t total = nq * nr * nm * nbc;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t bc = t % nbc;
        const int nu = (int)((t / nbc) % nm);
        const int64_t ir = t / (nbc * nm);  // i nr + r
        const int64_t i = ir / nr;
        const cd* Sr = S + ir * nm * nbc + bc;  // S[i, r, sa, bc]
        const cd* e = E1 + (i * nm + nu) * nm;  // E1[i, nu, sa]
        cd acc = {0.0, 0.0};
        for (int sa = 0; sa < nm; ++sa) acc = cfmac(e[sa], Sr[sa * nbc], acc);
        T[t] = acc;
    }
}

hipError_t launch_v3_fold(const cd* S, int64_t nq, int nr, int nm, const cd* E1, cd* T,
                          hipStream_t s) {
    const int64_t total = nq * nr * (int64_t)nm * nm * nm;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(v3_fold_kernel, dim3(grid_n(total, 256)), dim3(256), 0, s, S, nq, nr, nm, E1,
                       T);
    return hipGetLastError();
}

__global__ void v3_rot1_kernel(const cd* X, int64_t nqp, int nm, const cd* E2, cd* Y) {
    const int64_t m3 = (int64_t)nm * nm * nm;
    const int64_t total = nqp * m3;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(t % nm);
        const int nu2 = (int)((t / nm) % nm);
        const int nu = (int)((t / ((int64_t)nm * nm)) % nm);
        const int64_t j = t / m3;
        const cd* x = X + j * m3 + (int64_t)nu * nm * nm + c;  // X[j, nu, b, c]
        const cd* e = E2 + (j * nm + nu2) * nm;                 // E2[j, nu', b]
        cd acc = {0.0, 0.0};
        for (int b = 0; b < nm; ++b) acc = cfmac(e[b], x[(int64_t)b * nm], acc);
        Y[t] = acc;
    }
}

hipError_t launch_v3_rot1(const cd* X, int64_t nqp, int nm, const cd* E2, cd* Y, hipStream_t s) {
    const int64_t total = nqp * (int64_t)nm * nm * nm;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(v3_rot1_kernel, dim3(grid_n(total, 256)), dim3(256), 0, s, X, nqp, nm, E2, Y);
    return hipGetLastError();
}

__global__ void v3_rot2_kernel(const cd* Y, int64_t nqp, int nm, const cd* E3, cd* V) {
    const int64_t m3 = (int64_t)nm * nm * nm;
    const int64_t total = nqp * m3;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int nu3 = (int)(t % nm);
        const int64_t r = t / nm;  // (j nm + nu) nm + nu'
        const int64_t j = t / m3;
        const cd* y = Y + r * nm;                 // Y[j, nu, nu', c]
        const cd* e = E3 + (j * nm + nu3) * nm;   // E3[j, nu'', c]
        cd acc = {0.0, 0.0};
        for (int c = 0; c < nm; ++c) acc = cfmac(e[c], y[c], acc);
        V[t] = acc;
    }
}

hipError_t launch_v3_rot2(const cd* Y, int64_t nqp, int nm, const cd* E3, cd* V, hipStream_t s) {
    const int64_t total = nqp * (int64_t)nm * nm * nm;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(v3_rot2_kernel, dim3(grid_n(total, 256)), dim3(256), 0, s, Y, nqp, nm, E3, V);
    return hipGetLastError();
}

}  // namespace phx
