// Batched form: one persistent kernel drains a work queue of (system, state,
// q tile) tasks over many independent systems of different sizes.
//
// Each task forms X[q, sa*nW + b] = sum_Rp e^{i2pi q.Rp} F[Rp, sa*nW + b] for
// the tile's 16*TQ q points in FP32 on v_mfma_f32_16x16x4f32 (4 waves, TN
// column tiles of 16 per wave, as many column passes as the system needs), keeps
// the whole X tile in LDS, then applies the U_{k+q} and phonon rotations (FP32)
// and accumulates the smeared rate terms (FP64) into partial[state, q tile].
// (TQ, TN) is chosen per system by the autotuner.
#include "batched.hpp"

namespace phx {

template <int TQ, int TN>
__device__ void batched_tile(const SysDesc& d, int st, int qt, char* smem) {
    constexpr int BQ = 16 * TQ;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int W = 2 * d.rmax + 1;
    const int nW = d.nW, nm = d.nm, ldf = d.nc_pad;
    cd* sAx = reinterpret_cast<cd*>(smem);                       // [BQ][3][W]
    int* sRp = reinterpret_cast<int*>(sAx + BQ * 3 * W);         // [rp_pad]
    size_t off = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)d.rp_pad * sizeof(int);
    off = (off + 15) & ~(size_t)15;
    cf* sX = reinterpret_cast<cf*>(smem + off);                   // [BQ][nc_pad]
    cf* sY = sX + BQ * ldf;                                       // [BQ][kMBB][nm]
    int* sKq = reinterpret_cast<int*>(sY + BQ * kMBB * nm);       // [BQ]
    double* sRed = reinterpret_cast<double*>(sKq + BQ + (BQ & 1)); // [4]

    const int64_t qt0 = (int64_t)qt * BQ;
    const Mesh mesh = d.mesh;
    for (int i = tid; i < BQ * 3 * W; i += 256) {
        const int ql = i / (3 * W);
        const int dd = (i / W) % 3;
        const int r = i % W - d.rmax;
        const int64_t q = qt0 + ql;
        cd v = {0.0, 0.0};
        if (q < d.nq) {
            int i0, i1, i2;
            mesh_triple(q, mesh, i0, i1, i2);
            const int id = dd == 0 ? i0 : (dd == 1 ? i1 : i2);
            const int N = dd == 0 ? mesh.n0 : (dd == 1 ? mesh.n1 : mesh.n2);
            int t = (id * r) % N;
            if (t < 0) t += N;
            v = expi2pi((double)t / N);
        }
        sAx[i] = v;
    }
    const int zero_packed = d.rmax | (d.rmax << 8) | (d.rmax << 16);
    for (int i = tid; i < d.rp_pad; i += 256) sRp[i] = i < d.n_rp ? d.rp_packed[i] : zero_packed;
    __syncthreads();

    const cf* Fst = d.F + (int64_t)st * d.rp_pad * ldf;
    for (int c0 = 0; c0 < ldf; c0 += 64 * TN) {
        f4 cr[TQ][TN], ci[TQ][TN];
#pragma unroll
        for (int i = 0; i < TQ; ++i)
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                cr[i][t] = f4{0, 0, 0, 0};
                ci[i][t] = f4{0, 0, 0, 0};
            }
        const int colbase = c0 + wave * TN * 16 + li;
        for (int k0 = 0; k0 < d.rp_pad; k0 += 4) {
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
                    cr[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bv[t].x, cr[i][t], 0, 0, 0);
                    ci[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bv[t].y, ci[i][t], 0, 0, 0);
                }
#pragma unroll
            for (int i = 0; i < TQ; ++i)
#pragma unroll
                for (int t = 0; t < TN; ++t) {
                    cr[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[i], bv[t].y, cr[i][t], 0, 0, 0);
                    ci[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], bv[t].x, ci[i][t], 0, 0, 0);
                }
        }
        // f32 MFMA result v of lane group lg is tile row 4*lg + v
#pragma unroll
        for (int i = 0; i < TQ; ++i)
#pragma unroll
            for (int t = 0; t < TN; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    sX[(16 * i + 4 * lg + v) * ldf + colbase + t * 16] = cf{cr[i][t][v], ci[i][t][v]};
    }

    const int kmesh = d.st_kmesh[st];
    const int nband = d.st_band[st];
    const int mlo = d.st_mlo[st], mhi = d.st_mhi[st];
    int k0i, k1i, k2i;
    mesh_triple(kmesh, mesh, k0i, k1i, k2i);
    if (tid < BQ) {
        const int64_t q = qt0 + tid;
        int kq = -1;
        if (q < d.nq) {
            int q0, q1, q2;
            mesh_triple(q, mesh, q0, q1, q2);
            kq = (int)mesh_linear((k0i + q0) % mesh.n0, (k1i + q1) % mesh.n1, (k2i + q2) % mesh.n2,
                                  mesh);
        }
        sKq[tid] = kq;
    }
    __syncthreads();
    const double eps_n = d.eps[(int64_t)kmesh * nW + nband];
    const double inv_s2 = 1.0 / (d.sigma * d.sigma);
    double gacc = 0.0;
    for (int m0 = mlo; m0 <= mhi; m0 += kMBB) {
        const int nmb = min(kMBB, mhi - m0 + 1);
        for (int it = tid; it < BQ * nmb * nm; it += 256) {
            const int c = it / (nmb * nm);
            const int r = it - c * nmb * nm;
            const int mb = r / nm, sa = r - mb * nm;
            const int kq = sKq[c];
            float yr = 0.f, yi = 0.f;
            if (kq >= 0) {
                const cf* Xr = sX + c * ldf + sa * nW;
                const cd* Um = d.U + ((int64_t)kq * nW + m0 + mb) * nW;  // eigenvector m
                for (int b = 0; b < nW; ++b) {
                    const cf x = Xr[b];
                    const cd u = Um[b];
                    const float ur = (float)u.x, ui = (float)u.y;
                    yr = fmaf(x.x, ur, fmaf(-x.y, ui, yr));
                    yi = fmaf(x.x, ui, fmaf(x.y, ur, yi));
                }
            }
            sY[(c * kMBB + mb) * nm + sa] = cf{yr, yi};
        }
        __syncthreads();
        for (int it = tid; it < BQ * nmb * nm; it += 256) {
            const int c = it / (nmb * nm);
            const int r = it - c * nmb * nm;
            const int mb = r / nm, nu = r - mb * nm;
            const int kq = sKq[c];
            if (kq < 0) continue;
            const int64_t q = qt0 + c;
            const cf* Yr = sY + (c * kMBB + mb) * nm;
            const cd* Eq = d.E + (q * nm + nu) * nm;
            float zr = 0.f, zi = 0.f;
            for (int sa = 0; sa < nm; ++sa) {
                const cd e = Eq[sa];
                const float er = (float)e.x, ei = (float)e.y;
                const cf y = Yr[sa];
                zr = fmaf(er, y.x, fmaf(-ei, y.y, zr));
                zi = fmaf(er, y.y, fmaf(ei, y.x, zi));
            }
            const int m = m0 + mb;
            const double x = eps_n - d.eps[(int64_t)kq * nW + m];
            const double fm = d.focc[(int64_t)kq * nW + m];
            const double w = d.omega[q * nm + nu], nbq = d.nb[q * nm + nu];
            const double y1 = x - w, y2 = x + w;
            const double g1 = exp(-y1 * y1 * inv_s2), g2 = exp(-y2 * y2 * inv_s2);
            const double z2 = (double)zr * zr + (double)zi * zi;
            gacc += z2 * ((nbq + 1.0 - fm) * g1 + (nbq + fm) * g2);
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) gacc += __shfl_xor(gacc, o, 64);
    if (lane == 0) sRed[wave] = gacc;
    __syncthreads();
    if (tid == 0) d.partial[(int64_t)st * d.n_qtiles + qt] = (sRed[0] + sRed[1]) + (sRed[2] + sRed[3]);
    __syncthreads();
}

// Every work-group loops: take the next task index from the queue head, run
// it, stop when the queue is exhausted (every wave reaches the exit).
__global__ __launch_bounds__(256, 1) void batched_rates_kernel(const SysDesc* __restrict__ sys,
                                                               const BTask* __restrict__ tasks,
                                                               int n_tasks, int* head) {
    extern __shared__ char smem_raw[];
    __shared__ int s_task;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(head, 1);
        __syncthreads();
        const int t = s_task;
        __syncthreads();
        if (t >= n_tasks) break;
        const BTask tk = tasks[t];
        const SysDesc& d = sys[tk.sys];
        switch (d.tq * 100 + d.tn) {
            case 101: batched_tile<1, 1>(d, tk.state, tk.qtile, smem_raw); break;
            case 102: batched_tile<1, 2>(d, tk.state, tk.qtile, smem_raw); break;
            case 104: batched_tile<1, 4>(d, tk.state, tk.qtile, smem_raw); break;
            case 201: batched_tile<2, 1>(d, tk.state, tk.qtile, smem_raw); break;
            case 202: batched_tile<2, 2>(d, tk.state, tk.qtile, smem_raw); break;
            case 204: batched_tile<2, 4>(d, tk.state, tk.qtile, smem_raw); break;
            default: break;
        }
    }
}

bool batched_tile_supported(int tq, int tn) {
    return (tq == 1 || tq == 2) && (tn == 1 || tn == 2 || tn == 4);
}

size_t batched_lds(int tq, int rmax, int rp_pad, int nc_pad, int nm) {
    const int BQ = 16 * tq, W = 2 * rmax + 1;
    size_t shm = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)rp_pad * sizeof(int);
    shm = (shm + 15) & ~(size_t)15;
    shm += (size_t)BQ * nc_pad * sizeof(cf) + (size_t)BQ * kMBB * nm * sizeof(cf);
    shm += (size_t)(BQ + 1) * sizeof(int) + 8;
    shm = (shm + 7) & ~(size_t)7;
    shm += 4 * sizeof(double);
    return shm;
}

static size_t g_lds_set = 0;

hipError_t prepare_batched_rates(size_t lds) {
    if (lds > 160 * 1024 - 64) return hipErrorInvalidValue;
    if (lds <= g_lds_set) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)batched_rates_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) g_lds_set = lds;
    return e;
}

hipError_t launch_batched_rates(const SysDesc* sys, const BTask* tasks, int n_tasks, int* head,
                                int n_wg, size_t lds, hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    hipError_t e = prepare_batched_rates(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batched_rates_kernel, dim3(n_wg), dim3(256), lds, s, sys, tasks, n_tasks,
                       head);
    return hipGetLastError();
}

}  // namespace phx
