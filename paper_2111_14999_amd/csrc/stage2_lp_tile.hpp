// Device code shared by the reduced-precision rate kernels: BF16 splitting and
// MFMA helpers, and the fused stage-2 + rotation + rate tile that both the
// one-system launch (a grid of (q tile, state) work-groups) and the persistent
// multi-system kernel of the batched form (a queue of tasks) run.
#pragma once

#include "kernels.hpp"
#include "lowp.hpp"

namespace phx {

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
// Shared-memory slots of the rate tile besides its dynamic LDS block.
// ---------------------------------------------------------------------------
constexpr int kLpMaxCQ = 8;  // q rows per rotation chunk, TQ <= 2
struct LpShared {
    double red[4];
    double wq[kLpMaxCQ];
    int kq[kLpMaxCQ];
    int q[kLpMaxCQ];
};

// ---------------------------------------------------------------------------
// Fused stage 2 + rotations + rate terms, reduced precision: the work of one
// (state, q tile) task.  Same work decomposition as the FP64 kernel: one state x
// 16*TQ q per work-group, 4 waves with TN column tiles each.  Accumulator row of lane
// group lg, result v is 4*lg + v; the rotation works in four chunks c = lg
// (tile rows 4c .. 4c+3), in FP32 on the VALU.
// ---------------------------------------------------------------------------
template <int PREC, int TQ, int TN>
__device__ __forceinline__ void stage2_lp_tile(const RateArgsLP& a, int st, int qt, char* smem_raw,
                                               LpShared& sh) {
    constexpr int BQ = 16 * TQ;
    constexpr int CQ = 4 * TQ;
    static_assert(CQ <= kLpMaxCQ, "rotation chunk larger than the shared slots");
    constexpr int NP = PREC == PHOEBE_BF16X3 ? 2 : (PREC == PHOEBE_BF16X6 ? 3 : 1);
    const int W = 2 * a.rmax + 1;
    const int nW = a.nW, nm = a.nm;
    cd* sAx = reinterpret_cast<cd*>(smem_raw);                // [BQ][3][W]
    int* sRp = reinterpret_cast<int*>(sAx + BQ * 3 * W);      // [rp_pad]
    size_t off = (size_t)BQ * 3 * W * sizeof(cd) + (size_t)a.rp_pad * sizeof(int);
    off = (off + 15) & ~(size_t)15;
    cf* sX = reinterpret_cast<cf*>(smem_raw + off);            // [CQ][nc_pad]
    cf* sY = sX + CQ * a.nc_pad;                               // [CQ][MB][nm]
    // with a.stage, a rotation chunk's operands are staged once (coalesced) instead
    // of read per item: U_{k+q} rows of the pass' final bands and E_q of the chunk's
    // q points (FP32)
    const bool stg = a.stage != 0;
    cf* sU = sY + CQ * kMBLP * nm;                             // [CQ][MB][nW]
    cf* sE = sU + (stg ? CQ * kMBLP * nW : 0);                 // [CQ][nm][nm]
    double* sRed = sh.red;
    int* sKq = sh.kq;
    int* sQ = sh.q;
    double* sWq = sh.wq;

    // wave index marked uniform: the stores of the work-group's result below are
    // made by the whole of wave 0 (one value), not under a branch on the thread id
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lg = lane >> 4;
    int64_t qbeg = 0, qcount = a.nq_mesh;
    if (a.q_off) {
        const int row = a.st_row[st];
        qbeg = a.q_off[row];
        qcount = a.q_off[row + 1] - qbeg;
    }
    const int64_t qt0 = (int64_t)qt * BQ;
    if (__builtin_amdgcn_readfirstlane(qt0 >= qcount ? 1 : 0)) {  // the same for every lane
        if (wave == 0) a.partial[(int64_t)st * a.n_qtiles + qt] = 0.0;
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
        // B fragments of step k+4 are loaded while the MFMAs of step k run
        cf bv[TN];
        {
            const cf* Fr = Fst + (int64_t)lg * ldf + colbase;
#pragma unroll
            for (int t = 0; t < TN; ++t) bv[t] = Fr[t * 16];
        }
        for (int k0 = 0; k0 < a.rp_pad; k0 += 4) {
            const int k = k0 + lg;
            const int pk = sRp[k];
            const int p0 = pk & 255, p1 = (pk >> 8) & 255, p2 = (pk >> 16) & 255;
            cf bn[TN];
            const bool more = k0 + 4 < a.rp_pad;
            if (more) {
                const cf* Fr = Fst + (int64_t)(k + 4) * ldf + colbase;
#pragma unroll
                for (int t = 0; t < TN; ++t) bn[t] = Fr[t * 16];
            }
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
            if (more) {
#pragma unroll
                for (int t = 0; t < TN; ++t) bv[t] = bn[t];
            }
        }
    } else {
        using P = Pairs<PREC>;
        const int64_t per = (int64_t)a.rp_pad * a.nc_pad;
        const uint16_t* Fst = reinterpret_cast<const uint16_t*>(a.F) + (int64_t)st * 2 * NP * per;
        // The A fragments (phase pieces) are the same for the four waves: the
        // work-group forms each once per K step into LDS (double-buffered,
        // [buf][piece][re, im][i][lane] slots of 8 BF16), TPS threads per slot.
        s8v* sAf = reinterpret_cast<s8v*>(sE + (stg ? CQ * nm * nm : 0));
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
        // the chunk's E_q and the first pass' U_{k+q} rows (zero rows where the q is
        // beyond the list: no item reads them)
        auto stage_u = [&](int m0) {
            if (!stg) return;
            const int nmb = min(kMBLP, mhi - m0 + 1);
            for (int i = tid; i < CQ * nmb * nW; i += 256) {
                const int cc = i / (nmb * nW);
                const int r = i - cc * nmb * nW;
                const int mb = r / nW, b = r - mb * nW;
                const int kq = sKq[cc];
                cf v = {0.f, 0.f};
                if (kq >= 0) {
                    const cd u = a.U[((int64_t)kq * nW + m0 + mb) * nW + b];  // eigenvector m
                    v = cf{(float)u.x, (float)u.y};
                }
                sU[(cc * kMBLP + mb) * nW + b] = v;
            }
        };
        for (int i = tid; stg && i < CQ * nm * nm; i += 256) {
            const int cc = i / (nm * nm);
            const int r = i - cc * nm * nm;
            const int kq = sKq[cc];
            cf v = {0.f, 0.f};
            if (kq >= 0) {
                const cd e = a.E[(int64_t)sQ[cc] * nm * nm + r];
                v = cf{(float)e.x, (float)e.y};
            }
            sE[i] = v;
        }
        stage_u(mlo);
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
                    if (stg) {
                        const cf* Ur = sU + (cc * kMBLP + mb) * nW;
                        for (int b = 0; b < nW; ++b) {
                            const cf x = Xr[b];
                            const cf u = Ur[b];
                            yr = fmaf(x.x, u.x, fmaf(-x.y, u.y, yr));
                            yi = fmaf(x.x, u.y, fmaf(x.y, u.x, yi));
                        }
                    } else {
                        const cd* Um = a.U + ((int64_t)kq * nW + m0 + mb) * nW;  // eigenvector m
                        for (int b = 0; b < nW; ++b) {
                            const cf x = Xr[b];
                            const cd u = Um[b];
                            const float ur = (float)u.x, ui = (float)u.y;
                            yr = fmaf(x.x, ur, fmaf(-x.y, ui, yr));
                            yi = fmaf(x.x, ui, fmaf(x.y, ur, yi));
                        }
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
                const int m = m0 + mb;
                const double x = eps_n - a.eps[(int64_t)kq * nW + m];
                const double w = a.omega[q * nm + nu];
                const double y1 = x - w, y2 = x + w;
                // both Gaussians underflow to exactly 0 beyond 27.5 sigma: the term is 0
                if (fabs(y1) > 27.5 * a.sigma && fabs(y2) > 27.5 * a.sigma) continue;
                const cf* Yr = sY + (cc * kMBLP + mb) * nm;
                float zr = 0.f, zi = 0.f;
                if (stg) {
                    const cf* Er = sE + (cc * nm + nu) * nm;
                    for (int sa = 0; sa < nm; ++sa) {
                        const cf e = Er[sa];
                        const cf y = Yr[sa];
                        zr = fmaf(e.x, y.x, fmaf(-e.y, y.y, zr));
                        zi = fmaf(e.x, y.y, fmaf(e.y, y.x, zi));
                    }
                } else {
                    const cd* Eq = a.E + (q * nm + nu) * nm;
                    for (int sa = 0; sa < nm; ++sa) {
                        const cd e = Eq[sa];
                        const float er = (float)e.x, ei = (float)e.y;
                        const cf y = Yr[sa];
                        zr = fmaf(er, y.x, fmaf(-ei, y.y, zr));
                        zi = fmaf(er, y.y, fmaf(ei, y.x, zi));
                    }
                }
                const double fm = a.focc[(int64_t)kq * nW + m];
                const double nbq = a.nb[q * nm + nu];
                const double g1 = exp(-y1 * y1 * inv_s2), g2 = exp(-y2 * y2 * inv_s2);
                const double z2 = (double)zr * zr + (double)zi * zi;
                gacc += sWq[cc] * z2 * ((nbq + 1.0 - fm) * g1 + (nbq + fm) * g2);
            }
            // the next pass' U_{k+q} rows (this pass' Y loop, their only reader, is done)
            if (m0 + kMBLP <= mhi) stage_u(m0 + kMBLP);
            __syncthreads();
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) gacc += __shfl_xor(gacc, o, 64);
    if (lane == 0) sRed[wave] = gacc;
    __syncthreads();
    if (wave == 0)
        a.partial[(int64_t)st * a.n_qtiles + qt] = (sRed[0] + sRed[1]) + (sRed[2] + sRed[3]);
}

}  // namespace phx
