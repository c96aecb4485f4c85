// Coupling rotations and the scattering-rate sum on gfx950.
//
// The rate path evaluates, for each kept state (k, n) and each q of the mesh
// (or of an explicit list), the sum over Rp of the fixed-k precomputation
// F(k, Rp) = sum_Re e^{i2pi k.Re} U_k^dagger g(Re, Rp) (the Kokkos-section
// precompute with the k-side rotation folded in) on MFMA, rotates the result
// by U_{k+q} and by the scaled phonon eigenvectors, and accumulates the
// smeared rate terms; g(k, q) is never written to memory.
#include "kernels.hpp"

namespace phx {

static inline int grid1(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535 * 16) g = 65535 * 16;
    if (g < 1) g = 1;
    return (int)g;
}

// ---------------------------------------------------------------------------
// F[st, r, sa*nW + b] = sum_a conj(U_k[a, n]) G[kb, r, sa, a, b]
// ---------------------------------------------------------------------------
__global__ void fold_uk_kernel(const cd* __restrict__ G, int64_t ldg, const cd* __restrict__ U,
                               const int32_t* st_krow, int row0, const int32_t* st_kmesh,
                               const int32_t* st_band, int nst, int n_rp, int nm, int nW,
                               int rp_pad, int nc_pad, cd* __restrict__ F) {
    const int64_t per = (int64_t)rp_pad * nc_pad;
    const int64_t total = (int64_t)nst * per;
    const int nc = nm * nW;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int st = (int)(t / per);
        const int64_t o = t - st * per;
        const int r = (int)(o / nc_pad);
        const int c = (int)(o - (int64_t)r * nc_pad);
        cd acc = {0.0, 0.0};
        if (r < n_rp && c < nc) {
            const int sa = c / nW, b = c - sa * nW;
            const int n = st_band[st];
            const cd* Uk = U + (int64_t)st_kmesh[st] * nW * nW;
            const cd* Gk = G + (int64_t)(st_krow[st] - row0) * ldg + ((int64_t)r * nm + sa) * nW * nW + b;
            for (int a = 0; a < nW; ++a) acc = cfmac(Uk[a * nW + n], Gk[a * nW], acc);
        }
        F[t] = acc;
    }
}

hipError_t launch_fold_uk(const cd* G, int64_t ldg, const cd* U, const int32_t* st_krow,
                          int row0, const int32_t* st_kmesh, const int32_t* st_band, int nst, int n_rp,
                          int nm, int nW, int rp_pad, int nc_pad, cd* F, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    hipLaunchKernelGGL(fold_uk_kernel, dim3(grid1((int64_t)nst * rp_pad * nc_pad, 256)), dim3(256),
                       0, s, G, ldg, U, st_krow, row0, st_kmesh, st_band, nst, n_rp, nm, nW, rp_pad,
                       nc_pad, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused stage 2 + rotations + rate terms.
//
// Work-group = 4 waves = one state x BQ = 16*WQ q points.  Waves are arranged
// WQ (q row tiles) x WC (column groups); each wave holds TNW 16-column tiles
// of X[q, sa*nW + b] = sum_Rp e^{i2pi q.Rp} F[Rp, sa*nW + b] in MFMA
// accumulators.  The phase of (q, Rp) is the product of three per-axis
// factors e^{i2pi (i_d R_d mod N_d)/N_d} kept in LDS for the tile's q points.
//
// The rotation runs in two chunks of 8 rows per row tile: the chunk's X goes
// to LDS, then each (q, m) item forms Y[sa] = sum_b X[q, sa, b] U_{k+q}[b, m],
// Z[nu] = sum_sa E_q[sa, nu] Y[sa] and the rate terms
//   |Z|^2 [(n+1-f) G(x - w) + (n+f) G(x + w)],  G(y) = exp(-y^2/sigma^2),
// x = eps_nk - eps_{m,k+q}.  Final bands outside [mlo, mhi] are skipped: their
// Gaussians underflow to exactly zero in FP64 for every mode.
// ---------------------------------------------------------------------------
template <int WQ, int TNW, int NMX>
__global__ __launch_bounds__(256, 1) void stage2_rates_kernel(RateArgs a) {
    constexpr int BQ = 16 * WQ;
    constexpr int CQ = 8 * WQ;
    extern __shared__ char smem_raw[];
    const int W = 2 * a.rmax + 1;
    cd* sAx = reinterpret_cast<cd*>(smem_raw);               // [BQ][3][W]
    int* sRp = reinterpret_cast<int*>(sAx + BQ * 3 * W);     // [rp_pad]
    size_t off = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)a.rp_pad * sizeof(int);
    off = (off + 15) & ~(size_t)15;
    cd* sX = reinterpret_cast<cd*>(smem_raw + off);           // [CQ][nc_pad]
    __shared__ double sRed[4];

    const int st = blockIdx.y;
    const int qt = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wq = wave % WQ, wc = wave / WQ;
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

    // per-axis phase factors of the tile's q points
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

    // ---- stage 2 on MFMA ----
    d4 cr[TNW], ci[TNW];
#pragma unroll
    for (int t = 0; t < TNW; ++t) {
        cr[t] = d4{0, 0, 0, 0};
        ci[t] = d4{0, 0, 0, 0};
    }
    const cd* Fst = a.F + (int64_t)st * a.rp_pad * a.nc_pad;
    const int qlocal = wq * 16 + li;
    const cd* ax0 = sAx + qlocal * 3 * W;
    const cd* ax1 = ax0 + W;
    const cd* ax2 = ax1 + W;
    const int colbase = wc * TNW * 16 + li;
    const int ldf = a.nc_pad;
    cd bc[TNW];
    {
        const cd* Fr = Fst + (int64_t)lg * ldf + colbase;
#pragma unroll
        for (int t = 0; t < TNW; ++t) bc[t] = Fr[t * 16];
    }
    for (int k0 = 0; k0 < a.rp_pad; k0 += 4) {
        const int k = k0 + lg;
        const int pk = sRp[k];
        const cd ph = cmul(cmul(ax0[pk & 255], ax1[(pk >> 8) & 255]), ax2[(pk >> 16) & 255]);
        const double ar = ph.x, ai = ph.y, nai = -ph.y;
        cd bn[TNW];
        const bool more = k0 + 4 < a.rp_pad;
        if (more) {
            const cd* Fr = Fst + (int64_t)(k + 4) * ldf + colbase;
#pragma unroll
            for (int t = 0; t < TNW; ++t) bn[t] = Fr[t * 16];
        }
#pragma unroll
        for (int t = 0; t < TNW; ++t) {
            cr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bc[t].x, cr[t], 0, 0, 0);
            cr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai, bc[t].y, cr[t], 0, 0, 0);
            ci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bc[t].y, ci[t], 0, 0, 0);
            ci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bc[t].x, ci[t], 0, 0, 0);
        }
        if (more) {
#pragma unroll
            for (int t = 0; t < TNW; ++t) bc[t] = bn[t];
        }
    }

    // ---- rotations and rate terms ----
    const int kmesh = a.st_kmesh[st];
    const int nband = a.st_band[st];
    const int mlo = a.st_mlo[st], mhi = a.st_mhi[st];
    const int n_m = mhi - mlo + 1;
    const int nW = a.nW, nm = a.nm;
    int k0i, k1i, k2i;
    mesh_triple(kmesh, mesh, k0i, k1i, k2i);
    const double eps_n = a.eps[(int64_t)kmesh * nW + nband];
    const double inv_s2 = 1.0 / (a.sigma * a.sigma);
    double gacc = 0.0;
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
        __syncthreads();
        // result v of lane group lg is tile row lg + 4v: this chunk holds rows
        // 8ch .. 8ch+7, i.e. v = 2ch and 2ch+1 of every lane
#pragma unroll
        for (int t = 0; t < TNW; ++t)
#pragma unroll
            for (int vv = 0; vv < 2; ++vv) {
                const int v = 2 * ch + vv;
                const int qr = wq * 8 + lg + 4 * vv;
                sX[qr * ldf + colbase + t * 16] = cd{cr[t][v], ci[t][v]};
            }
        __syncthreads();
        if (n_m <= 0) continue;
        for (int it = tid; it < CQ * n_m; it += 256) {
            const int qc = it / n_m;
            const int m = mlo + (it - qc * n_m);
            const int qloc = (qc / 8) * 16 + 8 * ch + (qc % 8);
            const int64_t j = qt0 + qloc;
            if (j >= qcount) continue;
            const int64_t q = a.q_idx ? (int64_t)a.q_idx[qbeg + j] : j;
            const double wq_ = a.q_w ? a.q_w[qbeg + j] : 1.0;
            int q0, q1, q2;
            mesh_triple(q, mesh, q0, q1, q2);
            const int64_t kq = mesh_linear((k0i + q0) % mesh.n0, (k1i + q1) % mesh.n1,
                                           (k2i + q2) % mesh.n2, mesh);
            const cd* Xq = sX + qc * ldf;
            const cd* Uc = a.U + kq * nW * nW + m;
            cd Y[NMX];
#pragma unroll
            for (int s = 0; s < NMX; ++s) Y[s] = cd{0.0, 0.0};
            for (int b = 0; b < nW; ++b) {
                const cd u = Uc[(int64_t)b * nW];
#pragma unroll
                for (int s = 0; s < NMX; ++s)
                    if (s < nm) Y[s] = cfma(Xq[s * nW + b], u, Y[s]);
            }
            const double x = eps_n - a.eps[kq * nW + m];
            const double fm = a.focc[kq * nW + m];
            const cd* Eq = a.E + q * nm * nm;
            const double* wv = a.omega + q * nm;
            const double* nv = a.nb + q * nm;
            double tsum = 0.0;
            for (int nu = 0; nu < nm; ++nu) {
                cd z = {0.0, 0.0};
#pragma unroll
                for (int s = 0; s < NMX; ++s)
                    if (s < nm) z = cfma(Eq[s * nm + nu], Y[s], z);
                const double w = wv[nu], nbq = nv[nu];
                const double y1 = x - w, y2 = x + w;
                const double g1 = exp(-y1 * y1 * inv_s2), g2 = exp(-y2 * y2 * inv_s2);
                tsum += cabs2(z) * ((nbq + 1.0 - fm) * g1 + (nbq + fm) * g2);
            }
            gacc += wq_ * tsum;
        }
    }
    // fixed-order reduction of the work-group's partial sum
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) gacc += __shfl_xor(gacc, o, 64);
    if (lane == 0) sRed[wave] = gacc;
    __syncthreads();
    if (tid == 0)
        a.partial[(int64_t)st * a.n_qtiles + qt] = (sRed[0] + sRed[1]) + (sRed[2] + sRed[3]);
}

template <int WQ, int TNW, int NMX>
static hipError_t go_stage2(const RateArgs& a, int nst, hipStream_t s) {
    constexpr int BQ = 16 * WQ, CQ = 8 * WQ;
    const int W = 2 * a.rmax + 1;
    size_t shm = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)a.rp_pad * sizeof(int);
    shm = (shm + 15) & ~(size_t)15;
    shm += (size_t)CQ * a.nc_pad * sizeof(cd);
    if (shm > 160 * 1024 - 64) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)stage2_rates_kernel<WQ, TNW, NMX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    for (int s0 = 0; s0 < nst; s0 += 65535) {
        const int ns = nst - s0 < 65535 ? nst - s0 : 65535;
        RateArgs b = a;
        b.F = a.F + (int64_t)s0 * a.rp_pad * a.nc_pad;
        b.st_kmesh += s0;
        b.st_band += s0;
        b.st_row += s0;
        b.st_mlo += s0;
        b.st_mhi += s0;
        b.partial = a.partial + (int64_t)s0 * a.n_qtiles;
        hipLaunchKernelGGL((stage2_rates_kernel<WQ, TNW, NMX>), dim3(a.n_qtiles, ns), dim3(256),
                           shm, s, b);
    }
    return hipGetLastError();
}

// Column layout: nc = nm*nW split into 16-wide tiles; nc_pad = 16 * WC * TNW.
int stage2_config(int nm, int nW, int* wq_out, int* tnw_out) {
    const int nt = (nm * nW + 15) / 16;
    if (nt <= 16) {
        static const int opts[] = {1, 2, 3, 4, 6, 8, 12, 15, 16};
        for (int o : opts)
            if (o >= nt) {
                *wq_out = 4;
                *tnw_out = o;
                return 16 * o;
            }
    }
    if (nt <= 32) {  // WQ = 2, WC = 2
        const int t = (nt + 1) / 2;
        static const int opts[] = {9, 12, 16};
        for (int o : opts)
            if (o >= t) {
                *wq_out = 2;
                *tnw_out = o;
                return 16 * 2 * o;
            }
    }
    if (nt <= 64) {  // WQ = 1, WC = 4
        const int t = (nt + 3) / 4;
        static const int opts[] = {9, 12, 16};
        for (int o : opts)
            if (o >= t) {
                *wq_out = 1;
                *tnw_out = o;
                return 16 * 4 * o;
            }
    }
    return -1;
}

template <int NMX>
static hipError_t dispatch_stage2(const RateArgs& a, int nst, int wq, int tnw, hipStream_t s) {
#define PHX_CASE(WQv, TNWv) \
    if (wq == WQv && tnw == TNWv) return go_stage2<WQv, TNWv, NMX>(a, nst, s);
    PHX_CASE(4, 1) PHX_CASE(4, 2) PHX_CASE(4, 3) PHX_CASE(4, 4) PHX_CASE(4, 6) PHX_CASE(4, 8)
    PHX_CASE(4, 12) PHX_CASE(4, 15) PHX_CASE(4, 16)
    PHX_CASE(2, 9) PHX_CASE(2, 12) PHX_CASE(2, 16)
    PHX_CASE(1, 9) PHX_CASE(1, 12) PHX_CASE(1, 16)
#undef PHX_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_stage2_rates(const RateArgs& a, int nst, hipStream_t s) {
    if (nst <= 0 || a.n_qtiles <= 0) return hipSuccess;
    int wq = 0, tnw = 0;
    if (stage2_config(a.nm, a.nW, &wq, &tnw) != a.nc_pad) return hipErrorInvalidValue;
    if (a.nm <= 8) return dispatch_stage2<8>(a, nst, wq, tnw, s);
    if (a.nm <= 16) return dispatch_stage2<16>(a, nst, wq, tnw, s);
    if (a.nm <= 32) return dispatch_stage2<32>(a, nst, wq, tnw, s);
    return hipErrorInvalidValue;
}

__global__ void reduce_partials_kernel(const double* partial, int nst, int ntiles,
                                       const int32_t* st_row, const int32_t* st_band, int nW,
                                       double scale, double* gamma) {
    const int st = blockIdx.x * blockDim.x + threadIdx.x;
    if (st >= nst) return;
    const double* p = partial + (int64_t)st * ntiles;
    double acc = 0.0;
    for (int t = 0; t < ntiles; ++t) acc += p[t];
    gamma[(int64_t)st_row[st] * nW + st_band[st]] = scale * acc;
}

hipError_t launch_reduce_partials(const double* partial, int nst, int ntiles,
                                  const int32_t* st_row, const int32_t* st_band, int nW,
                                  double scale, double* gamma, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((nst + 127) / 128), dim3(128), 0, s, partial,
                       nst, ntiles, st_row, st_band, nW, scale, gamma);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// State lists of the rate path
// ---------------------------------------------------------------------------
// rowflag[a, n] = mask[kept[a], n]; optional copies to the caller's outputs.
__global__ void gather_rows_kernel(const uint8_t* mask, const int32_t* kept, int64_t rows, int nW,
                                   int32_t* rowflag, uint8_t* mask_out, int32_t* kept_out) {
    const int64_t total = rows * nW;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = t / nW;
        const int n = (int)(t - a * nW);
        const uint8_t v = mask[(int64_t)kept[a] * nW + n];
        rowflag[t] = v;
        if (mask_out) mask_out[t] = v;
        if (kept_out && n == 0) kept_out[a] = kept[a];
    }
}

hipError_t launch_gather_rows(const uint8_t* mask, const int32_t* kept, int64_t rows, int nW,
                              int32_t* rowflag, uint8_t* mask_out, int32_t* kept_out,
                              hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid1(rows * nW, 256)), dim3(256), 0, s, mask,
                       kept, rows, nW, rowflag, mask_out, kept_out);
    return hipGetLastError();
}

// From state ids (row*nW + band): the state's row, band, mesh k and the range
// of final bands whose Gaussians can be non-zero for some q and mode.
__global__ void build_states_kernel(const int32_t* ids, int nst, int nW, const int32_t* kept,
                                    const double* eps, const double* bmin, const double* bmax,
                                    const double* wmax, double cut, int32_t* st_row,
                                    int32_t* st_band, int32_t* st_kmesh, int32_t* st_mlo,
                                    int32_t* st_mhi) {
    const int st = blockIdx.x * blockDim.x + threadIdx.x;
    if (st >= nst) return;
    const int id = ids[st];
    const int row = id / nW, band = id - row * nW;
    const int km = kept[row];
    const double e = eps[(int64_t)km * nW + band];
    const double lo = e - *wmax - cut, hi = e + *wmax + cut;
    int mlo = nW, mhi = -1;
    for (int m = 0; m < nW; ++m) {
        if (bmax[m] >= lo && bmin[m] <= hi) {
            if (m < mlo) mlo = m;
            mhi = m;
        }
    }
    st_row[st] = row;
    st_band[st] = band;
    st_kmesh[st] = km;
    st_mlo[st] = mlo;
    st_mhi[st] = mhi;
}

hipError_t launch_build_states(const int32_t* ids, int nst, int nW, const int32_t* kept,
                               const double* eps, const double* bmin, const double* bmax,
                               const double* wmax, double cut, int32_t* st_row, int32_t* st_band,
                               int32_t* st_kmesh, int32_t* st_mlo, int32_t* st_mhi,
                               hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    hipLaunchKernelGGL(build_states_kernel, dim3((nst + 127) / 128), dim3(128), 0, s, ids, nst, nW,
                       kept, eps, bmin, bmax, wmax, cut, st_row, st_band, st_kmesh, st_mlo, st_mhi);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// interp_g helpers
// ---------------------------------------------------------------------------
// F[r, sa, n, b] = sum_a conj(U[a, n]) G[r, sa, a, b]
__global__ void fold_all_kernel(const cd* __restrict__ G, const cd* __restrict__ U, int n_rp,
                                int nm, int nW, cd* __restrict__ F) {
    const int64_t total = (int64_t)n_rp * nm * nW * nW;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nW);
        const int n = (int)((t / nW) % nW);
        const int64_t rs = t / ((int64_t)nW * nW);  // r*nm + sa
        const cd* Gp = G + rs * nW * nW + b;
        cd acc = {0.0, 0.0};
        for (int a = 0; a < nW; ++a) acc = cfmac(U[a * nW + n], Gp[a * nW], acc);
        F[t] = acc;
    }
}

hipError_t launch_fold_all(const cd* G, const cd* U, int n_rp, int nm, int nW, cd* F,
                           hipStream_t s) {
    hipLaunchKernelGGL(fold_all_kernel, dim3(grid1((int64_t)n_rp * nm * nW * nW, 256)), dim3(256),
                       0, s, G, U, n_rp, nm, nW, F);
    return hipGetLastError();
}

// g[q, nu, n, m] = sum_sa E[q, sa, nu] sum_b X[q, sa, n, b] Ukq[q, b, m]
__global__ void rotate_g_kernel(const cd* __restrict__ X, int64_t nq, const cd* __restrict__ Ukq,
                                const cd* __restrict__ E, int nW, int nm, cd* __restrict__ g) {
    const int64_t total = nq * nW * nW;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(t % nW);
        const int n = (int)((t / nW) % nW);
        const int64_t q = t / ((int64_t)nW * nW);
        const cd* Xq = X + q * nm * nW * nW;
        const cd* Uq = Ukq + q * nW * nW;
        const cd* Eq = E + q * nm * nm;
        cd Y[32];
        for (int sa = 0; sa < nm; ++sa) {
            cd acc = {0.0, 0.0};
            const cd* xr = Xq + ((int64_t)sa * nW + n) * nW;
            for (int b = 0; b < nW; ++b) acc = cfma(xr[b], Uq[b * nW + m], acc);
            Y[sa] = acc;
        }
        cd* go = g + q * nm * nW * nW;
        for (int nu = 0; nu < nm; ++nu) {
            cd z = {0.0, 0.0};
            for (int sa = 0; sa < nm; ++sa) z = cfma(Eq[sa * nm + nu], Y[sa], z);
            go[((int64_t)nu * nW + n) * nW + m] = z;
        }
    }
}

hipError_t launch_rotate_g(const cd* X, int64_t nq, const cd* Uk, const cd* Ukq, const cd* E,
                           int nW, int nm, cd* g, hipStream_t s) {
    (void)Uk;
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(rotate_g_kernel, dim3(grid1(nq * nW * nW, 128)), dim3(128), 0, s, X, nq,
                       Ukq, E, nW, nm, g);
    return hipGetLastError();
}

}  // namespace phx
