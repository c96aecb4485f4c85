// Coupling rotations and the scattering-rate sum on gfx950.
//
// The rate path evaluates, for each kept state (k, n) and each q of the mesh
// (or of an explicit list), the sum over Rp of the fixed-k precomputation
// F(k, Rp) = sum_Re e^{i2pi k.Re} U_k^dagger g(Re, Rp) (the Kokkos-section
// precompute with the k-side rotation folded in) on MFMA, rotates the result
// by U_{k+q} and by the scaled phonon eigenvectors, and accumulates the
// smeared rate terms; g(k, q) is never written to memory.
#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace phx {

static inline int grid1(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535 * 16) g = 65535 * 16;
    if (g < 1) g = 1;
    return (int)g;
}

// ---------------------------------------------------------------------------
// F[st, r, sa*cw + b] = sum_a conj(U_k[a, n]) G[kb, r, sa, a, b]   (U passed transposed)
// (cw = column width per mode index: nW for the direct sum, 16 for the
// factorised one, whose rate kernel keeps one mode index per MFMA tile)
// ---------------------------------------------------------------------------
__global__ void fold_uk_kernel(const cd* __restrict__ G, int64_t ldg, const cd* __restrict__ U,
                               const int32_t* st_krow, int row0, const int32_t* st_kmesh,
                               const int32_t* st_band, int nst, int n_rp, int nm, int nW, int cw,
                               int rp_pad, int nc_pad, cd* __restrict__ F) {
    const int64_t per = (int64_t)rp_pad * nc_pad;
    const int64_t total = (int64_t)nst * per;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int st = (int)(t / per);
        const int64_t o = t - st * per;
        const int r = (int)(o / nc_pad);
        const int c = (int)(o - (int64_t)r * nc_pad);
        const int sa = c / cw, b = c - sa * cw;
        cd acc = {0.0, 0.0};
        if (r < n_rp && sa < nm && b < nW) {
            const int n = st_band[st];
            const cd* Un = U + ((int64_t)st_kmesh[st] * nW + n) * nW;  // eigenvector n
            const cd* Gk = G + (int64_t)(st_krow[st] - row0) * ldg + ((int64_t)r * nm + sa) * nW * nW + b;
            for (int a = 0; a < nW; ++a) acc = cfmac(Un[a], Gk[a * nW], acc);
        }
        F[t] = acc;
    }
}

// Zero of the padding of F [nst, rp_pad, nc_pad] (elements of esize bytes): rows
// n_rp.. and columns ncol.. of every row; the rest is written by the fold.
__global__ void zero_fpad_kernel(char* F, int64_t nst, int rp_pad, int nc_pad, int n_rp, int ncol,
                                 int esize) {
    const int64_t pad_row = (int64_t)nc_pad - ncol;  // padded columns of a data row
    const int64_t per = (int64_t)n_rp * pad_row + (int64_t)(rp_pad - n_rp) * nc_pad;
    const int64_t total = nst * per;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t st = t / per, o = t - st * per;
        int64_t r, c;
        if (o < (int64_t)n_rp * pad_row) {
            r = o / pad_row;
            c = ncol + (o - r * pad_row);
        } else {
            const int64_t o2 = o - (int64_t)n_rp * pad_row;
            r = n_rp + o2 / nc_pad;
            c = o2 % nc_pad;
        }
        char* e = F + ((st * rp_pad + r) * nc_pad + c) * esize;
        for (int i = 0; i < esize; i += 4) *reinterpret_cast<uint32_t*>(e + i) = 0u;
    }
}

hipError_t launch_zero_fpad(void* F, int64_t nst, int rp_pad, int nc_pad, int n_rp, int ncol,
                            int esize, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    if (n_rp > rp_pad || ncol > nc_pad || esize % 4 != 0) return hipErrorInvalidValue;
    const int64_t per = (int64_t)n_rp * (nc_pad - ncol) + (int64_t)(rp_pad - n_rp) * nc_pad;
    if (per == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_fpad_kernel, dim3(grid1(nst * per, 256)), dim3(256), 0, s,
                       reinterpret_cast<char*>(F), nst, rp_pad, nc_pad, n_rp, ncol, esize);
    return hipGetLastError();
}

hipError_t launch_fold_uk(const cd* G, int64_t ldg, const cd* U, const int32_t* st_krow,
                          int row0, const int32_t* st_kmesh, const int32_t* st_band, int nst, int n_rp,
                          int nm, int nW, int cw, int rp_pad, int nc_pad, cd* F, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    if (cw < nW || (int64_t)cw * nm > nc_pad) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fold_uk_kernel, dim3(grid1((int64_t)nst * rp_pad * nc_pad, 256)), dim3(256),
                       0, s, G, ldg, U, st_krow, row0, st_kmesh, st_band, nst, n_rp, nm, nW, cw,
                       rp_pad, nc_pad, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused stage 2 + rotations + rate terms.
//
// Work-group = 4 waves = one state x BQ = 16*TQ q points.  Every wave holds the
// same TQ row tiles of 16 q and its own TN column tiles of 16 columns of
//   X[q, sa*nW + b] = sum_Rp e^{i2pi q.Rp} F[Rp, sa*nW + b],
// so nc_pad = 64*TN.  The phase of (q, Rp) is the product of three per-axis
// factors e^{i2pi (i_d R_d mod N_d)/N_d} kept in LDS for the tile's q points.
// MFMA f64 16x16x4 layouts: lane l holds A[l%16][l/16] and B[l/16][l%16];
// result v of lane l is row l/16 + 4v, column l%16.
//
// The rotation runs in four chunks (one per result index v, 4*TQ q rows):
// the chunk's X goes to LDS; threads over (q, m, sa) form
// Y[q, sa, m] = sum_b X[q, sa, b] U_{k+q}[b, m]; threads over (q, m, nu) form
// Z = sum_sa E_q[sa, nu] Y[q, sa, m] and the rate terms
//   |Z|^2 [(n+1-f) G(x - w) + (n+f) G(x + w)],  G(y) = exp(-y^2/sigma^2),
// x = eps_nk - eps_{m,k+q}.  Final bands outside [mlo, mhi] are skipped: their
// Gaussians underflow to exactly zero in FP64 for every mode.
// ---------------------------------------------------------------------------
constexpr int kMB = 8;  // final bands per rotation pass

template <int TQ, int TN>
__global__ __launch_bounds__(256, (TN >= 12 ? 1 : 2)) void stage2_rates_kernel(RateArgs a) {
    constexpr int BQ = 16 * TQ;
    constexpr int CQ = 4 * TQ;  // q rows per rotation chunk
    extern __shared__ char smem_raw[];
    const int W = 2 * a.rmax + 1;
    const int nW = a.nW, nm = a.nm;
    cd* sAx = reinterpret_cast<cd*>(smem_raw);               // [BQ][3][W]
    int* sRp = reinterpret_cast<int*>(sAx + BQ * 3 * W);     // [rp_pad]
    size_t off = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)a.rp_pad * sizeof(int);
    off = (off + 15) & ~(size_t)15;
    cd* sX = reinterpret_cast<cd*>(smem_raw + off);           // [CQ][nc_pad]
    cd* sY = sX + CQ * a.nc_pad;                              // [CQ][kMB][nm]
    // per-term outputs (terms or linewidth, never both): [CQ][kMB][nm], summed
    // over the bands of a pass in order by one thread per (q, mode)
    double* sT = reinterpret_cast<double*>(sY + CQ * kMB * nm);
    double* const tout = a.terms ? a.terms : a.lw;
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
    d4 cr[TQ][TN], ci[TQ][TN];
#pragma unroll
    for (int i = 0; i < TQ; ++i)
#pragma unroll
        for (int t = 0; t < TN; ++t) {
            cr[i][t] = d4{0, 0, 0, 0};
            ci[i][t] = d4{0, 0, 0, 0};
        }
    const cd* Fst = a.F + (int64_t)st * a.rp_pad * a.nc_pad;
    const int colbase = wave * TN * 16 + li;
    const int ldf = a.nc_pad;
    // B fragments of step k+4 are loaded while the MFMAs of step k run
    cd bc[TN];
    {
        const cd* Fr = Fst + (int64_t)lg * ldf + colbase;
#pragma unroll
        for (int t = 0; t < TN; ++t) bc[t] = Fr[t * 16];
    }
    for (int k0 = 0; k0 < a.rp_pad; k0 += 4) {
        const int k = k0 + lg;
        const int pk = sRp[k];
        const int p0 = pk & 255, p1 = (pk >> 8) & 255, p2 = (pk >> 16) & 255;
        cd bn[TN];
        const bool more = k0 + 4 < a.rp_pad;
        if (more) {
            const cd* Fr = Fst + (int64_t)(k + 4) * ldf + colbase;
#pragma unroll
            for (int t = 0; t < TN; ++t) bn[t] = Fr[t * 16];
        }
        double ar[TQ], ai[TQ];
#pragma unroll
        for (int i = 0; i < TQ; ++i) {
            const cd* ax = sAx + (16 * i + li) * 3 * W;
            const cd ph = cmul(cmul(ax[p0], ax[W + p1]), ax[2 * W + p2]);
            ar[i] = ph.x;
            ai[i] = ph.y;
        }
#pragma unroll
        for (int i = 0; i < TQ; ++i)
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                cr[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bc[t].x, cr[i][t], 0, 0, 0);
                ci[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bc[t].y, ci[i][t], 0, 0, 0);
            }
#pragma unroll
        for (int i = 0; i < TQ; ++i)
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                cr[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bc[t].y, cr[i][t], 0, 0, 0);
                ci[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bc[t].x, ci[i][t], 0, 0, 0);
            }
        if (more) {
#pragma unroll
            for (int t = 0; t < TN; ++t) bc[t] = bn[t];
        }
    }

    // ---- rotations and rate terms ----
    const int kmesh = a.st_kmesh[st];
    const int nband = a.st_band[st];
    const int mlo = a.st_mlo[st], mhi = a.st_mhi[st];
    int k0i, k1i, k2i;
    mesh_triple(kmesh, mesh, k0i, k1i, k2i);
    const double eps_n = a.eps[(int64_t)kmesh * nW + nband];
    const double inv_s2 = 1.0 / (a.sigma * a.sigma);
    double gacc = 0.0;
    // extensions (FP64): v_nk for adaptive widths, f (1 - f) / kT for the linewidth
    double vn[3] = {0.0, 0.0, 0.0};
    if (a.vel)
        for (int d = 0; d < 3; ++d) vn[d] = a.vel[((int64_t)kmesh * nW + nband) * 3 + d];
    double mdf = 0.0;
    if (a.lw) {
        const double fn = a.focc[(int64_t)kmesh * nW + nband];
        mdf = fn * (1.0 - fn) * a.inv_kT;
    }
    const cd* Ukn = a.U + ((int64_t)kmesh * nW + nband) * nW;  // U_k column n (transposed table)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        __syncthreads();
        // chunk row c = 4*i + lg holds tile row 16*i + lg + 4*v
#pragma unroll
        for (int i = 0; i < TQ; ++i)
#pragma unroll
            for (int t = 0; t < TN; ++t)
                sX[(4 * i + lg) * ldf + colbase + t * 16] = cd{cr[i][t][v], ci[i][t][v]};
        if (tid < CQ) {
            const int c = tid;
            const int qloc = 16 * (c >> 2) + (c & 3) + 4 * v;
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
            sKq[c] = kq;
            sQ[c] = q;
            sWq[c] = w;
        }
        __syncthreads();
        for (int m0 = mlo; m0 <= mhi; m0 += kMB) {
            const int nmb = min(kMB, mhi - m0 + 1);
            // Y[c, mb, sa] = sum_b X[c, sa*nW + b] U_{k+q}[b, m0 + mb]
            for (int it = tid; it < CQ * nmb * nm; it += 256) {
                const int c = it / (nmb * nm);
                const int r = it - c * nmb * nm;
                const int mb = r / nm, sa = r - mb * nm;
                const int kq = sKq[c];
                cd y = {0.0, 0.0};
                if (kq >= 0) {
                    const cd* Xr = sX + c * ldf + sa * nW;
                    const cd* Um = a.U + ((int64_t)kq * nW + m0 + mb) * nW;  // eigenvector m
                    for (int b = 0; b < nW; ++b) y = cfma(Xr[b], Um[b], y);
                }
                sY[(c * kMB + mb) * nm + sa] = y;
            }
            __syncthreads();
            // Z[c, mb, nu] = sum_sa E_q[sa, nu] Y[c, mb, sa]; rate terms
            for (int it = tid; it < CQ * nmb * nm; it += 256) {
                const int c = it / (nmb * nm);
                const int r = it - c * nmb * nm;
                const int mb = r / nm, nu = r - mb * nm;
                const int kq = sKq[c];
                if (kq < 0) continue;
                const int64_t q = sQ[c];
                const cd* Yr = sY + (c * kMB + mb) * nm;
                const cd* Eq = a.E + (q * nm + nu) * nm;
                cd z = {0.0, 0.0};
                for (int sa = 0; sa < nm; ++sa) z = cfma(Eq[sa], Yr[sa], z);
                const int m = m0 + mb;
                if (a.Lpol) {  // + i L(q, nu) [U_k^dagger U_{k+q}]_{n m}
                    const cd* Ukq = a.U + ((int64_t)kq * nW + m) * nW;
                    cd o = {0.0, 0.0};
                    for (int b = 0; b < nW; ++b) o = cfmac(Ukn[b], Ukq[b], o);
                    const cd l = a.Lpol[q * nm + nu];
                    z.x -= l.x * o.y + l.y * o.x;
                    z.y += l.x * o.x - l.y * o.y;
                }
                double is2 = inv_s2, wt = 1.0;
                if (a.vel) {  // adaptive width of the transition
                    const double* vm = a.vel + ((int64_t)kq * nW + m) * 3;
                    double s2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        const double t = a.ad_c[d] * (vn[d] - vm[d]);
                        s2 += t * t;
                    }
                    const double sg = fmax(a.sigma, sqrt(s2));
                    is2 = 1.0 / (sg * sg);
                    wt = 1.0 / sg;
                }
                const double x = eps_n - a.eps[(int64_t)kq * nW + m];
                const double fm = a.focc[(int64_t)kq * nW + m];
                const double w = a.omega[q * nm + nu], nbq = a.nb[q * nm + nu];
                const double y1 = x - w, y2 = x + w;
                const double g1 = wt * exp(-y1 * y1 * is2), g2 = wt * exp(-y2 * y2 * is2);
                const double z2 = cabs2(z);
                const double term = z2 * ((nbq + 1.0 - fm) * g1 + (nbq + fm) * g2);
                gacc += sWq[c] * term;
                if (tout) sT[(c * kMB + mb) * nm + nu] = a.terms ? a.terms_scale * term : mdf * z2 * g1;
            }
            __syncthreads();
            if (tout) {  // (state, q) belongs to this work-group alone: plain adds, fixed order
                for (int it = tid; it < CQ * nm; it += 256) {
                    const int c = it / nm, nu = it - c * nm;
                    if (sKq[c] < 0) continue;
                    double sum = 0.0;
                    for (int mb = 0; mb < nmb; ++mb) sum += sT[(c * kMB + mb) * nm + nu];
                    tout[((int64_t)st * a.nq_mesh + sQ[c]) * nm + nu] += sum;
                }
                __syncthreads();
            }
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

static size_t stage2_lds(int TQ, int rmax, int rp_pad, int nc_pad, int nm, bool per_term) {
    const int BQ = 16 * TQ, CQ = 4 * TQ, W = 2 * rmax + 1;
    size_t shm = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)rp_pad * sizeof(int);
    shm = (shm + 15) & ~(size_t)15;
    shm += (size_t)CQ * nc_pad * sizeof(cd) + (size_t)CQ * kMB * nm * sizeof(cd);
    if (per_term) shm += (size_t)CQ * kMB * nm * sizeof(double);
    return shm;
}

template <int TQ, int TN>
static hipError_t go_stage2(const RateArgs& a, int nst, hipStream_t s) {
    if (a.terms && a.lw) return hipErrorInvalidValue;
    const size_t shm = stage2_lds(TQ, a.rmax, a.rp_pad, a.nc_pad, a.nm, a.terms || a.lw);
    if (shm > 160 * 1024 - 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)stage2_rates_kernel<TQ, TN>,
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
        if (a.terms) b.terms = a.terms + (int64_t)s0 * a.nq_mesh * a.nm;
        if (a.lw) b.lw = a.lw + (int64_t)s0 * a.nq_mesh * a.nm;
        hipLaunchKernelGGL((stage2_rates_kernel<TQ, TN>), dim3(a.n_qtiles, ns), dim3(256), shm, s,
                           b);
    }
    return hipGetLastError();
}

// Column tiling of nc = nm*nW: 4 waves x TN tiles of 16 (nc_pad = 64 TN) and
// TQ row tiles of 16 q per work-group.  Returns nc_pad and the q tile BQ.
int stage2_config(int nm, int nW, int* tq_out, int* tn_out) {
    const int nt = (nm * nW + 15) / 16;
    static const int tns[] = {1, 2, 3, 4, 6, 8, 12, 16};
    for (int tn : tns) {
        if (4 * tn >= nt) {
            *tn_out = tn;
            *tq_out = tn <= 2 ? 4 : (tn <= 4 ? 2 : 1);
            return 64 * tn;
        }
    }
    return -1;
}

hipError_t launch_stage2_rates(const RateArgs& a, int nst, hipStream_t s) {
    if (nst <= 0 || a.n_qtiles <= 0) return hipSuccess;
    int tq = 0, tn = 0;
    if (stage2_config(a.nm, a.nW, &tq, &tn) != a.nc_pad) return hipErrorInvalidValue;
#define PHX_CASE(TQv, TNv) \
    if (tq == TQv && tn == TNv) return go_stage2<TQv, TNv>(a, nst, s);
    PHX_CASE(4, 1) PHX_CASE(4, 2) PHX_CASE(2, 3) PHX_CASE(2, 4) PHX_CASE(1, 6) PHX_CASE(1, 8)
    PHX_CASE(1, 12) PHX_CASE(1, 16)
#undef PHX_CASE
    return hipErrorInvalidValue;
}

// one wave per state: lane j sums tiles j, j + 64, ... in order, then a fixed
// butterfly over the wave (the same order on every call)
__global__ void reduce_partials_kernel(const double* partial, int nst, int ntiles,
                                       const int32_t* st_row, const int32_t* st_band, int nW,
                                       double scale, double* gamma) {
    const int st = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (st >= nst) return;
    const double* p = partial + (int64_t)st * ntiles;
    double acc = 0.0;
#pragma unroll 4
    for (int t = lane; t < ntiles; t += 64) acc += p[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) gamma[(int64_t)st_row[st] * nW + st_band[st]] = scale * acc;
}

hipError_t launch_reduce_partials(const double* partial, int nst, int ntiles,
                                  const int32_t* st_row, const int32_t* st_band, int nW,
                                  double scale, double* gamma, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((nst + 3) / 4), dim3(256), 0, s, partial,
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
// Smearing weights of the rate sum for each state and (q, mode):
//   D[st, q, nu] = scale sum_{m in [mlo, mhi]} [(n+1-f_m) e^{-(x-w)^2/s^2} + (n+f_m) e^{-(x+w)^2/s^2}],
// x = eps_nk - eps_{m,k+q}, w = hbar omega_{q nu}; 0 for modes below omega_min.
// With it the rate term of (q, nu) is |g|^2 x D, so terms / D is a smooth
// |g|^2 average the learned proposal fits.
// ---------------------------------------------------------------------------
__global__ void delta_weights_kernel(int nst, int64_t N, Mesh mesh, const int32_t* st_kmesh,
                                     const int32_t* st_band, const int32_t* st_mlo,
                                     const int32_t* st_mhi, const double* eps, const double* focc,
                                     const double* omega, const double* nb, int nW, int nm,
                                     double sigma, double omega_min, double scale, double* D) {
    const int64_t total = (int64_t)nst * N;
    const double inv_s2 = 1.0 / (sigma * sigma);
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int st = (int)(t / N);
        const int64_t q = t - (int64_t)st * N;
        const int km = st_kmesh[st];
        int k0, k1, k2, q0, q1, q2;
        mesh_triple(km, mesh, k0, k1, k2);
        mesh_triple(q, mesh, q0, q1, q2);
        const int64_t kq =
            mesh_linear((k0 + q0) % mesh.n0, (k1 + q1) % mesh.n1, (k2 + q2) % mesh.n2, mesh);
        const double en = eps[(int64_t)km * nW + st_band[st]];
        double* Dq = D + t * nm;
        for (int nu = 0; nu < nm; ++nu) {
            const double w = omega[q * nm + nu];
            double acc = 0.0;
            if (w >= omega_min && w > 0.0) {
                const double n = nb[q * nm + nu];
                for (int m = st_mlo[st]; m <= st_mhi[st]; ++m) {
                    const double x = en - eps[kq * nW + m];
                    const double f = focc[kq * nW + m];
                    const double y1 = x - w, y2 = x + w;
                    acc += (n + 1.0 - f) * exp(-y1 * y1 * inv_s2) + (n + f) * exp(-y2 * y2 * inv_s2);
                }
            }
            Dq[nu] = scale * acc;
        }
    }
}

hipError_t launch_delta_weights(int nst, int64_t N, Mesh mesh, const int32_t* st_kmesh,
                                const int32_t* st_band, const int32_t* st_mlo,
                                const int32_t* st_mhi, const double* eps, const double* focc,
                                const double* omega, const double* nb, int nW, int nm, double sigma,
                                double omega_min, double scale, double* D, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    hipLaunchKernelGGL(delta_weights_kernel, dim3(grid1((int64_t)nst * N, 256)), dim3(256), 0, s,
                       nst, N, mesh, st_kmesh, st_band, st_mlo, st_mhi, eps, focc, omega, nb, nW,
                       nm, sigma, omega_min, scale, D);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// interp_g helpers
// ---------------------------------------------------------------------------
// F[r, sa, n, b] = sum_a conj(U[a, n]) G[r, sa, a, b]
// F rows (one per Rp) are ldf elements apart (ldf >= nm nW^2)
__global__ void fold_all_kernel(const cd* __restrict__ G, const cd* __restrict__ U, int n_rp,
                                int nm, int nW, cd* __restrict__ F, int64_t ldf) {
    const int64_t nc = (int64_t)nm * nW * nW;
    const int64_t total = (int64_t)n_rp * nc;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(t % nW);
        const int n = (int)((t / nW) % nW);
        const int64_t rs = t / ((int64_t)nW * nW);  // r*nm + sa
        const cd* Gp = G + rs * nW * nW + b;
        cd acc = {0.0, 0.0};
        for (int a = 0; a < nW; ++a) acc = cfmac(U[a * nW + n], Gp[a * nW], acc);
        const int64_t r = t / nc;
        F[r * ldf + (t - r * nc)] = acc;
    }
}

hipError_t launch_fold_all(const cd* G, const cd* U, int n_rp, int nm, int nW, cd* F,
                           hipStream_t s, int64_t ldf) {
    const int64_t nc = (int64_t)nm * nW * nW;
    if (ldf < 0) ldf = nc;
    if (ldf < nc) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fold_all_kernel, dim3(grid1((int64_t)n_rp * nc, 256)), dim3(256), 0, s, G,
                       U, n_rp, nm, nW, F, ldf);
    return hipGetLastError();
}

// g[q, nu, n, m] = sum_sa E[q, nu, sa] sum_b X[q, sa, n, b] Ukq[q, b, m]
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
            for (int sa = 0; sa < nm; ++sa) z = cfma(Eq[nu * nm + sa], Y[sa], z);
            go[((int64_t)nu * nW + n) * nW + m] = z;
        }
    }
}

// The same rotation with one work-group per q (nW <= 16): X[q] and E_q are staged
// in LDS once; thread (n, m) holds U_{k+q}[:, m] and Y[sa] = sum_b X[q, sa, n, b]
// U[b, m] for every sa in registers and writes g[q, nu, n, m] (m fastest).  The
// sums run in the same order as above.
template <int NMX>
__global__ __launch_bounds__(256) void rotate_g_lds_kernel(const cd* __restrict__ X,
                                                           const cd* __restrict__ Ukq,
                                                           const cd* __restrict__ E, int nW,
                                                           int nm, cd* __restrict__ g) {
    extern __shared__ char smem_raw[];
    const int nc = nm * nW * nW;
    cd* sX = reinterpret_cast<cd*>(smem_raw);  // [nm][nW][nW]
    cd* sE = sX + nc;                          // [nu][sa]
    const int64_t q = blockIdx.x;
    const int tid = threadIdx.x;
    const cd* Xq = X + q * nc;
    for (int i = tid; i < nc; i += blockDim.x) sX[i] = Xq[i];
    const cd* Eq = E + q * nm * nm;
    for (int i = tid; i < nm * nm; i += blockDim.x) sE[i] = Eq[i];
    __syncthreads();
    if (tid >= nW * nW) return;
    const int n = tid / nW, m = tid - n * nW;
    const cd* Uq = Ukq + q * nW * nW;
    cd u[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) u[b] = b < nW ? Uq[b * nW + m] : cd{0.0, 0.0};
    cd Y[NMX];
#pragma unroll
    for (int sa = 0; sa < NMX; ++sa) {
        cd acc = {0.0, 0.0};
        if (sa < nm) {
            const cd* xr = sX + (sa * nW + n) * nW;
#pragma unroll
            for (int b = 0; b < 16; ++b)
                if (b < nW) acc = cfma(xr[b], u[b], acc);
        }
        Y[sa] = acc;
    }
    cd* go = g + q * nc + n * nW + m;
    for (int nu = 0; nu < nm; ++nu) {
        const cd* er = sE + nu * nm;
        cd z = {0.0, 0.0};
#pragma unroll
        for (int sa = 0; sa < NMX; ++sa)
            if (sa < nm) z = cfma(er[sa], Y[sa], z);
        go[(int64_t)nu * nW * nW] = z;
    }
}

// The rotation on FP64 MFMA (nW, nModes <= 16; indices padded to 16 with zeros),
// one work-group of four waves per q, wave w taking n = 4w .. 4w + 3.  Per n two
// 16 x 16 x 16 complex products, each four K steps of v_mfma_f64_16x16x4f64 for
// every real product:
//   W^T[b, nu] = sum_sa X[q, sa, n, b] E[q, nu, sa]      (A: lane (i, j) X[4s + j][n][i])
//   g[nu, n, m] = sum_b W[nu, b] U_{k+q}[b, m]            (A: W, B: lane (i, j) U[4s + j][i])
// The first product leaves W[nu = i][b = j + 4v] in result v of lane (i, j), which is
// the A operand of K step s = v of the second: no data moves between the two.  g's
// row nu = j + 4v, column m = i: four 256-byte runs per store.  The sums are the
// same as the VALU kernels' up to the order of the additions.
__global__ __launch_bounds__(256) void rotate_g_mfma_kernel(const cd* __restrict__ X,
                                                            const cd* __restrict__ Ukq,
                                                            const cd* __restrict__ E, int nW,
                                                            int nm, cd* __restrict__ g) {
    const int64_t q = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t nc = (int64_t)nm * nW * nW;
    const cd* Xq = X + q * nc;
    const cd* Uq = Ukq + q * nW * nW;
    const cd* Eq = E + q * nm * nm;
    const cd z = {0.0, 0.0};
    cd e[4], u[4];  // B operands: E[nu = i][sa = 4s + j], U[b = 4s + j][m = i]
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + lg;
        e[s] = (li < nm && k < nm) ? Eq[li * nm + k] : z;
        u[s] = (k < nW && li < nW) ? Uq[k * nW + li] : z;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int n = 4 * wave + t;
        if (n >= nW) break;  // the same for the whole wave
        cd x[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int sa = 4 * s + lg;
            x[s] = (sa < nm && li < nW) ? Xq[((int64_t)sa * nW + n) * nW + li] : z;
        }
        d4 wr = {0, 0, 0, 0}, wi = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) cmfma_f64(wr, wi, x[s].x, x[s].y, e[s].x, e[s].y);
        d4 gr = {0, 0, 0, 0}, gi = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) cmfma_f64(gr, gi, wr[s], wi[s], u[s].x, u[s].y);
        cd* go = g + q * nc + (int64_t)n * nW + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int nu = lg + 4 * v;
            if (nu < nm && li < nW) go[(int64_t)nu * nW * nW] = cd{gr[v], gi[v]};
        }
    }
}

hipError_t launch_rotate_g(const cd* X, int64_t nq, const cd* Uk, const cd* Ukq, const cd* E,
                           int nW, int nm, cd* g, hipStream_t s) {
    (void)Uk;
    if (nq <= 0) return hipSuccess;
    if (nW <= 16 && nm <= 16 && nq <= 2147483647LL) {
        hipLaunchKernelGGL(rotate_g_mfma_kernel, dim3((unsigned)nq), dim3(256), 0, s, X, Ukq, E,
                           nW, nm, g);
        return hipGetLastError();
    }
    const size_t shm = ((size_t)nm * nW * nW + (size_t)nm * nm) * sizeof(cd);
    if (nW <= 16 && nm <= 32 && shm <= 160 * 1024 && nq <= 2147483647LL) {
        const int block = std::max(64, (nW * nW + 63) / 64 * 64);
        auto go = [&](auto nmx) {
            constexpr int NMX = decltype(nmx)::value;
            hipError_t e = hipFuncSetAttribute((const void*)rotate_g_lds_kernel<NMX>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(rotate_g_lds_kernel<NMX>, dim3((unsigned)nq), dim3(block), shm, s, X,
                               Ukq, E, nW, nm, g);
            return hipGetLastError();
        };
        if (nm <= 8) return go(std::integral_constant<int, 8>{});
        if (nm <= 16) return go(std::integral_constant<int, 16>{});
        return go(std::integral_constant<int, 32>{});
    }
    hipLaunchKernelGGL(rotate_g_kernel, dim3(grid1(nq * nW * nW, 128)), dim3(128), 0, s, X, nq,
                       Ukq, E, nW, nm, g);
    return hipGetLastError();
}

}  // namespace phx
