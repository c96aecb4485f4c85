// Stage 2 on a full q mesh, factorised over the three axes.
//
// On a full mesh the phase of (q, Rp) is the product of three per-axis
// factors, e^{i2pi q.Rp} = P0[q0, R0] P1[q1, R1] P2[q2, R2] with
// Pd[n, r] = e^{i2pi (n r mod N_d) / N_d}, so the sum over Rp of the fixed-k
// precomputation F(k, Rp) splits into three one-axis transforms
// (Electron Properties, interpolation of g; the Kokkos-section precompute at
// fixed k).  Rp is embedded in the box [-rmax, rmax]^3 (W = 2 rmax + 1 per
// axis) with zeros where the list has no vector:
//   T1[R0, R1, q2, c] = sum_R2 P2[q2, R2] F[R0, R1, R2, c]
//   T2[R0, q1, q2, c] = sum_R1 P1[q1, R1] T1[R0, R1, q2, c]
//   X [q0, q1, q2, c] = sum_R0 P0[q0, R0] T2[R0, q1, q2, c]
// The last transform runs on MFMA inside the rate kernel, one work-group per
// (state, q1, q2) line of N0 points, followed by the same rotations and
// smeared rate terms as the direct kernel; X never reaches memory.  The sum
// is the same as the direct one up to the order of the additions.
#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace phx {

static inline int gridm(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g > 65535 * 16) g = 65535 * 16;
    if (g < 1) g = 1;
    return (int)g;
}

// P[d][n, r] for the three axes, stored one after another ([N0 + N1 + N2, W])
__global__ void axis_phase_kernel(Mesh m, int rmax, cd* P) {
    const int W = 2 * rmax + 1;
    const int total = (m.n0 + m.n1 + m.n2) * W;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        const int row = t / W;
        const int r = t - row * W - rmax;
        int n = row, N = m.n0;
        if (n >= m.n0) {
            n -= m.n0;
            N = m.n1;
            if (n >= m.n1) {
                n -= m.n1;
                N = m.n2;
            }
        }
        int a = (int)(((int64_t)n * r) % N);
        if (a < 0) a += N;
        P[t] = expi2pi((double)a / N);
    }
}

hipError_t launch_axis_phases(Mesh m, int rmax, cd* P, hipStream_t s) {
    const int W = 2 * rmax + 1;
    hipLaunchKernelGGL(axis_phase_kernel, dim3(gridm((int64_t)(m.n0 + m.n1 + m.n2) * W, 256)),
                       dim3(256), 0, s, m, rmax, P);
    return hipGetLastError();
}

constexpr int kMaxW = 32;

// T1[st, p, q2, c] = sum_r P2[q2, r] F[st, box_rp[p W + r], c]   (p = (R0, R1))
// box_rp maps a box position to its row of F, or -1 where the list has no Rp.
// WT > 0 fixes the box width at compile time (the W inputs stay in registers);
// WT = 0 takes it from the argument.  C is the working type: cd (FP64) or cf
// (FP32 form: phases formed in FP64 and rounded once, FP32 accumulation).
template <int WT, class C>
__global__ __launch_bounds__(256) void axis2_kernel(const C* __restrict__ F, int rp_pad,
                                                    int nc_pad, const int32_t* __restrict__ box_rp,
                                                    int Wr, int N2, const cd* __restrict__ P2,
                                                    int nst, C* __restrict__ T1) {
    constexpr int NV = WT > 0 ? WT : kMaxW;
    const int W = WT > 0 ? WT : Wr;
    const int64_t total = (int64_t)nst * W * W * nc_pad;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(t % nc_pad);
        const int64_t sp = t / nc_pad;  // st * W^2 + p
        const int p = (int)(sp % (W * W));
        const int st = (int)(sp / (W * W));
        C v[NV];
#pragma unroll
        for (int r = 0; r < NV; ++r) {
            if (r < W) {
                const int row = box_rp[p * W + r];
                v[r] = row >= 0 ? F[((int64_t)st * rp_pad + row) * nc_pad + c] : C{0, 0};
            }
        }
        C* out = T1 + sp * N2 * nc_pad + c;
        for (int q = 0; q < N2; ++q) {
            const cd* Pq = P2 + q * W;
            C acc = {0, 0};
#pragma unroll
            for (int r = 0; r < NV; ++r)
                if (r < W) acc = cfma(to_c<C>(Pq[r]), v[r], acc);
            out[(int64_t)q * nc_pad] = acc;
        }
    }
}

// out[o, n, i] = sum_r P[n, r] in[o, r, i]   (i < inner, contiguous); here
// o = (st, R0), n = q1 and i = (q2, column).  With line_any set, the output of a
// (st, line = q1 N2 + q2) whose flag is 0 is not formed: the line kernel never
// reads it.
template <int WT, class C>
__global__ __launch_bounds__(256) void axis_mid_kernel(const C* __restrict__ in, int64_t n_outer,
                                                       int Wr, int64_t inner, int N,
                                                       const cd* __restrict__ P,
                                                       const uint32_t* __restrict__ line_any,
                                                       int nc, C* __restrict__ out) {
    constexpr int NV = WT > 0 ? WT : kMaxW;
    const int W = WT > 0 ? WT : Wr;
    const int64_t total = n_outer * inner;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t % inner;
        const int64_t o = t / inner;
        C v[NV];
        const C* src = in + o * W * inner + i;
#pragma unroll
        for (int r = 0; r < NV; ++r)
            if (r < W) v[r] = src[(int64_t)r * inner];
        C* dst = out + o * N * inner + i;
        const int64_t n2 = inner / nc, q2 = i / nc;
        const uint32_t* fl = line_any ? line_any + (o / W) * N * n2 + q2 : nullptr;
        for (int n = 0; n < N; ++n) {
            if (fl && !fl[n * n2]) continue;
            const cd* Pn = P + n * W;
            C acc = {0, 0};
#pragma unroll
            for (int r = 0; r < NV; ++r)
                if (r < W) acc = cfma(to_c<C>(Pn[r]), v[r], acc);
            dst[(int64_t)n * inner] = acc;
        }
    }
}

// Both Rp axes in one pass: a work-group takes one (state, R0, 64-column block),
// stages its F rows (R1, R2) in LDS and, for each q2 of its share, forms
//   T1[R1] = sum_R2 P2[q2, R2] F[st, box_rp[(R0 W + R1) W + R2], c]
// in registers, then T2[st, R0, q1 N2 + q2, c] = sum_R1 P1[q1, R1] T1[R1] for the
// live lines.  The sums run in the same order as axis2 then axis_mid, so the two
// routes agree bit for bit; T1 never goes through HBM.  Wave g of the work-group
// (64 lanes, one column each) takes q2 = g, g + kAxisWaves, ...  Eight waves
// share one slab and the kernel is compiled for six waves per SIMD (80 VGPRs), so
// that three work-groups (three FP64 slabs of a box 7 wide) fill a CU.
constexpr int kAxisWaves = 8;

template <int WT, class C>
__global__ __launch_bounds__(64 * kAxisWaves, 6) void axis_fused_kernel(const C* __restrict__ F, int rp_pad,
                                                         int nc_pad, const int32_t* __restrict__ box_rp,
                                                         Mesh m, const cd* __restrict__ P1,
                                                         const cd* __restrict__ P2,
                                                         const uint32_t* __restrict__ line_any,
                                                         int qsplit, C* __restrict__ T2) {
    constexpr int W = WT;
    extern __shared__ char smem_raw[];
    C* sF = reinterpret_cast<C*>(smem_raw);  // [W * W][64]
    const int ncb = nc_pad / 64;
    int64_t b = blockIdx.x;
    const int qs = (int)(b % qsplit);  // this work-group's share of the q2 values
    b /= qsplit;
    const int cb = (int)(b % ncb);
    b /= ncb;
    const int r0 = (int)(b % W);
    const int st = (int)(b / W);
    const int tid = threadIdx.x, cc = tid & 63, g = tid >> 6;
    const int c = cb * 64 + cc;
    const C* Fs = F + (int64_t)st * rp_pad * nc_pad + c;
    for (int i = g; i < W * W; i += kAxisWaves) {
        const int row = box_rp[r0 * W * W + i];
        st_vec(sF + i * 64 + cc, row >= 0 ? ld_vec(Fs + (int64_t)row * nc_pad) : C{0, 0});
    }
    __syncthreads();
    const int N1 = m.n1, N2 = m.n2, NL = N1 * N2;
    const uint32_t* fl = line_any + (int64_t)st * NL;
    C* out = T2 + ((int64_t)st * W + r0) * NL * nc_pad + c;
    for (int q2 = g + kAxisWaves * qs; q2 < N2; q2 += kAxisWaves * qsplit) {
        // the slab is read from LDS per q2, not held in registers across the loop
        asm volatile("" ::: "memory");
        C t1[W];
        const cd* Pq = P2 + q2 * W;
#pragma unroll
        for (int r1 = 0; r1 < W; ++r1) {
            C acc = {0, 0};
#pragma unroll
            for (int r2 = 0; r2 < W; ++r2)
                acc = cfma(to_c<C>(Pq[r2]), ld_vec(sF + (r1 * W + r2) * 64 + cc), acc);
            t1[r1] = acc;
        }
        for (int q1 = 0; q1 < N1; ++q1) {
            const int line = q1 * N2 + q2;
            if (!fl[line]) continue;
            const cd* Pn = P1 + q1 * W;
            C acc = {0, 0};
#pragma unroll
            for (int r1 = 0; r1 < W; ++r1) acc = cfma(to_c<C>(Pn[r1]), t1[r1], acc);
            st_vec(out + (int64_t)line * nc_pad, acc);
        }
    }
}

template <int WT, class C>
static hipError_t go_axes(const C* F, int rp_pad, int nc_pad, const int32_t* box_rp, int W,
                          Mesh m, const cd* P1, const cd* P2, int nst, const uint32_t* line_any,
                          C* T1, C* T2, hipStream_t s) {
    // one pass where the box is a compile-time width, the F slab fits 64 KB of LDS
    // and the columns come in 64-wide blocks
    if constexpr (WT > 0) {
        const size_t shm = (size_t)WT * WT * 64 * sizeof(C);
        if (line_any && shm <= 64 * 1024 && nc_pad % 64 == 0) {
            hipError_t e = hipFuncSetAttribute((const void*)axis_fused_kernel<WT, C>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            if (e != hipSuccess) return e;
            // a few states make few work-groups: split the q2 values of a slab over up to
            // ceil(N2 / waves) work-groups (each reloads the slab) until the grid fills the chip
            const int64_t base = (int64_t)nst * WT * (nc_pad / 64);
            const int qmax = (m.n2 + kAxisWaves - 1) / kAxisWaves;
            int qsplit = 1;
            while (qsplit < qmax && base * qsplit < 2048) ++qsplit;
            const int64_t groups = base * qsplit;
            if (groups > 2147483647LL) return hipErrorInvalidValue;
            hipLaunchKernelGGL((axis_fused_kernel<WT, C>), dim3((unsigned)groups), dim3(64 * kAxisWaves),
                               shm, s,
                               F, rp_pad, nc_pad, box_rp, m, P1, P2, line_any, qsplit, T2);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((axis2_kernel<WT, C>), dim3(gridm((int64_t)nst * W * W * nc_pad, 256)),
                       dim3(256), 0, s, F, rp_pad, nc_pad, box_rp, W, m.n2, P2, nst, T1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t inner = (int64_t)m.n2 * nc_pad;
    hipLaunchKernelGGL((axis_mid_kernel<WT, C>), dim3(gridm((int64_t)nst * W * inner, 256)),
                       dim3(256), 0, s, T1, (int64_t)nst * W, W, inner, m.n1, P1, line_any, nc_pad,
                       T2);
    return hipGetLastError();
}

template <class C>
static hipError_t axis_transforms(const C* F, int rp_pad, int nc_pad, const int32_t* box_rp,
                                  int rmax, Mesh m, const cd* P, int nst, const uint32_t* line_any,
                                  C* T1, C* T2, hipStream_t s) {
    const int W = 2 * rmax + 1;
    if (W > kMaxW) return hipErrorInvalidValue;
    if (nst <= 0) return hipSuccess;
    const cd* P1 = P + (int64_t)m.n0 * W;
    const cd* P2 = P1 + (int64_t)m.n1 * W;
    switch (W) {
        case 1: return go_axes<1, C>(F, rp_pad, nc_pad, box_rp, W, m, P1, P2, nst, line_any, T1, T2, s);
        case 3: return go_axes<3, C>(F, rp_pad, nc_pad, box_rp, W, m, P1, P2, nst, line_any, T1, T2, s);
        case 5: return go_axes<5, C>(F, rp_pad, nc_pad, box_rp, W, m, P1, P2, nst, line_any, T1, T2, s);
        case 7: return go_axes<7, C>(F, rp_pad, nc_pad, box_rp, W, m, P1, P2, nst, line_any, T1, T2, s);
        case 9: return go_axes<9, C>(F, rp_pad, nc_pad, box_rp, W, m, P1, P2, nst, line_any, T1, T2, s);
        default: return go_axes<0, C>(F, rp_pad, nc_pad, box_rp, W, m, P1, P2, nst, line_any, T1, T2, s);
    }
}

// The last axis written out, for g on the full mesh (interpolation):
//   X[(q0 - q0a) NL + line, c] = sum_R0 P0[q0, R0] T2[R0, line, c],  q0 in [q0a, q0b),
// X rows ldx elements apart, columns c < nc.  A thread takes one (line, c): it
// reads its W values of T2 once and writes one value per q0 (consecutive threads,
// consecutive c: coalesced).
template <int WT, class C>
__global__ __launch_bounds__(256) void axis0_out_kernel(const C* __restrict__ T2, int64_t NL,
                                                        int nc_pad, int nc, int Wr,
                                                        const cd* __restrict__ P0, int q0a, int q0b,
                                                        C* __restrict__ X, int64_t ldx) {
    constexpr int NV = WT > 0 ? WT : kMaxW;
    const int W = WT > 0 ? WT : Wr;
    const int64_t total = NL * nc;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t line = i / nc;
        const int c = (int)(i - line * nc);
        C v[NV];
#pragma unroll
        for (int r = 0; r < NV; ++r)
            if (r < W) v[r] = T2[((int64_t)r * NL + line) * nc_pad + c];
        for (int q0 = q0a; q0 < q0b; ++q0) {
            const cd* Pq = P0 + (int64_t)q0 * W;
            C acc = {0, 0};
#pragma unroll
            for (int r = 0; r < NV; ++r)
                if (r < W) acc = cfma(to_c<C>(Pq[r]), v[r], acc);
            X[((int64_t)(q0 - q0a) * NL + line) * ldx + c] = acc;
        }
    }
}

template <class C>
static hipError_t axis0_out(const C* T2, Mesh m, int nc_pad, int nc, int rmax, const cd* P,
                            int q0a, int q0b, C* X, int64_t ldx, hipStream_t s) {
    const int W = 2 * rmax + 1;
    if (W > kMaxW || nc > nc_pad || q0a < 0 || q0b > m.n0 || ldx < nc) return hipErrorInvalidValue;
    if (q0b <= q0a) return hipSuccess;
    const int64_t NL = (int64_t)m.n1 * m.n2;
    const dim3 g(gridm(NL * nc, 256)), b(256);
    switch (W) {
        case 1: hipLaunchKernelGGL((axis0_out_kernel<1, C>), g, b, 0, s, T2, NL, nc_pad, nc, W, P, q0a, q0b, X, ldx); break;
        case 3: hipLaunchKernelGGL((axis0_out_kernel<3, C>), g, b, 0, s, T2, NL, nc_pad, nc, W, P, q0a, q0b, X, ldx); break;
        case 5: hipLaunchKernelGGL((axis0_out_kernel<5, C>), g, b, 0, s, T2, NL, nc_pad, nc, W, P, q0a, q0b, X, ldx); break;
        case 7: hipLaunchKernelGGL((axis0_out_kernel<7, C>), g, b, 0, s, T2, NL, nc_pad, nc, W, P, q0a, q0b, X, ldx); break;
        case 9: hipLaunchKernelGGL((axis0_out_kernel<9, C>), g, b, 0, s, T2, NL, nc_pad, nc, W, P, q0a, q0b, X, ldx); break;
        default: hipLaunchKernelGGL((axis0_out_kernel<0, C>), g, b, 0, s, T2, NL, nc_pad, nc, W, P, q0a, q0b, X, ldx); break;
    }
    return hipGetLastError();
}

hipError_t launch_axis0_out(const cd* T2, Mesh m, int nc_pad, int nc, int rmax, const cd* P,
                            int q0a, int q0b, cd* X, int64_t ldx, hipStream_t s) {
    return axis0_out<cd>(T2, m, nc_pad, nc, rmax, P, q0a, q0b, X, ldx, s);
}
hipError_t launch_axis0_out_f32(const cf* T2, Mesh m, int nc_pad, int nc, int rmax, const cd* P,
                                int q0a, int q0b, cf* X, int64_t ldx, hipStream_t s) {
    return axis0_out<cf>(T2, m, nc_pad, nc, rmax, P, q0a, q0b, X, ldx, s);
}

// The last axis and the rotation of g on the full mesh in one pass (FP64, nW and
// nModes <= 16, box width WT <= 7): X never reaches memory.  A wave takes one band n
// of one line (q1, q2) and holds, in the A-operand layout of the rotation's first
// product, the line's T2 entries T2[R0, line, (sa, n, b)] for sa = 4s + j, b = i
// (lane (i, j), K step s).  For every q0 of the line it forms
//   X[q, sa, n, b] = sum_R0 P0[q0, R0] T2[R0, line, (sa, n, b)]
// in registers and runs the two chained products of rotate_g_mfma_kernel (E_q X,
// then that times U_{k+q}), writing g[q, nu, n, m].  Each complex product takes
// three real ones (Gauss: Ar Br, Ai Bi and (Ar + Ai)(Br + Bi)) instead of four.
// A work-group is four waves (bands 4p .. 4p + 3); the work-groups of one line are
// dealt to one XCD, so that line's E_q and U_{k+q} come from one L2.
//
// Every load and store is a buffer access over the one object it touches (a
// T2 row, E_q, U_{k+q}, g[q]); a lane outside the matrices (row or column beyond
// nModes or nW) gets an offset past the object's size, so the hardware range
// check returns zero or drops the store.  No access sits under a lane branch,
// which keeps the count of memory operations in flight fixed, so the compiler's
// waits name exact counts: E_q and U_{k+q} of the next q0 are issued at the top of
// each pass and first waited for after the current pass's X and its first product.
namespace {
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
constexpr int kOob = 0x7FFFFFF0;  // past every object below (each is < 2 GiB)
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
__device__ inline cd bld(__amdgpu_buffer_rsrc_t r, int off) {
    const u4v v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return __builtin_bit_cast(cd, v);
}
__device__ inline void bst(__amdgpu_buffer_rsrc_t r, int off, cd v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, v), r, off, 0, 0);
}
struct Bop {  // a complex B operand and the sum of its parts
    double r, i, s;
};
__device__ inline Bop bop(cd v) { return Bop{v.x, v.y, v.x + v.y}; }
// one K step of a complex product by Gauss's three real products
__device__ inline void gauss_step(d4& t1, d4& t2, d4& t3, double ar, double ai, const Bop& b) {
    t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, b.r, t1, 0, 0, 0);
    t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, b.i, t2, 0, 0, 0);
    t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, b.s, t3, 0, 0, 0);
}
}  // namespace

template <int WT>
__global__ __launch_bounds__(256, 2) void axis0_rotate_kernel(
    const cd* __restrict__ T2, int64_t NL, int ncp, int N0, const cd* __restrict__ P0,
    const cd* __restrict__ E, const cd* __restrict__ Ukq, int nW, int nm, int nwg_line,
    cd* __restrict__ g) {
    const int64_t id = blockIdx.x;
    const int xcd = (int)(id & 7);
    const int64_t j = id >> 3;
    const int64_t line = (j / nwg_line) * 8 + xcd;
    const int part = (int)(j % nwg_line);
    if (line >= NL) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lg = lane >> 4;
    const int n = 4 * part + wave;
    if (n >= nW) return;  // the same for the whole wave; no barriers below
    const int64_t nc = (int64_t)nm * nW * nW;
    // lane offsets (bytes) into a T2 row / E_q / U_{k+q} for K step s, into g[q] for row v
    int ot[4], oe[4], ou[4], og[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + lg;
        ot[s] = (k < nm && li < nW) ? ((k * nW + n) * nW + li) * 16 : kOob;
        oe[s] = (li < nm && k < nm) ? (li * nm + k) * 16 : kOob;
        ou[s] = (k < nW && li < nW) ? (k * nW + li) * 16 : kOob;
        og[s] = (k < nm && li < nW) ? (k * nW * nW + n * nW + li) * 16 : kOob;  // nu = lg + 4v
    }
    cd t2[WT][4];
#pragma unroll
    for (int r = 0; r < WT; ++r) {
        const auto rt = rsrc(T2 + ((int64_t)r * NL + line) * ncp, (int64_t)ncp * 16);
#pragma unroll
        for (int s = 0; s < 4; ++s) t2[r][s] = bld(rt, ot[s]);
    }
    auto load_eu = [&](int q0, cd (&e)[4], cd (&u)[4]) {
        const int64_t q = (int64_t)q0 * NL + line;
        const auto re = rsrc(E + q * nm * nm, (int64_t)nm * nm * 16);
        const auto ru = rsrc(Ukq + q * nW * nW, (int64_t)nW * nW * 16);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            e[s] = bld(re, oe[s]);
            u[s] = bld(ru, ou[s]);
        }
    };
    Bop be[4], bu[4];
    {
        cd e[4], u[4];
        load_eu(0, e, u);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            be[s] = bop(e[s]);
            bu[s] = bop(u[s]);
        }
    }
    // T2 and the first operands are in registers before the loop starts, so that the
    // loop's own waits count only its own accesses
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    for (int q0 = 0; q0 < N0; ++q0) {
        cd en[4], un[4];
        load_eu(q0 + 1 < N0 ? q0 + 1 : q0, en, un);  // the last pass reloads its own
        const cd* Pq = P0 + (int64_t)q0 * WT;
        cd x[4] = {};
#pragma unroll
        for (int r = 0; r < WT; ++r) {
            const cd p = Pq[r];
#pragma unroll
            for (int s = 0; s < 4; ++s) x[s] = cfma(p, t2[r][s], x[s]);
        }
        d4 t1 = {0, 0, 0, 0}, tb = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) gauss_step(t1, tb, t3, x[s].x, x[s].y, be[s]);
        const d4 wr = t1 - tb, wi = t3 - t1 - tb;
        t1 = d4{0, 0, 0, 0};
        tb = d4{0, 0, 0, 0};
        t3 = d4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) gauss_step(t1, tb, t3, wr[s], wi[s], bu[s]);
        const d4 gr = t1 - tb, gi = t3 - t1 - tb;
        const auto rg = rsrc(g + ((int64_t)q0 * NL + line) * nc, nc * 16);
#pragma unroll
        for (int v = 0; v < 4; ++v) bst(rg, og[v], cd{gr[v], gi[v]});
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            be[s] = bop(en[s]);
            bu[s] = bop(un[s]);
        }
    }
}

bool axis0_rotate_supported(int rmax, int nW, int nm) {
    const int W = 2 * rmax + 1;
    return nW <= 16 && nm <= 16 && (W == 1 || W == 3 || W == 5 || W == 7);
}

hipError_t launch_axis0_rotate(const cd* T2, Mesh m, int ncp, int rmax, const cd* P,
                               const cd* E, const cd* Ukq, int nW, int nm, cd* g, hipStream_t s) {
    const int W = 2 * rmax + 1;
    if (!axis0_rotate_supported(rmax, nW, nm)) return hipErrorInvalidValue;
    const int64_t NL = (int64_t)m.n1 * m.n2;
    const int nwg_line = (nW + 3) / 4;
    const int64_t groups = (NL + 7) / 8 * 8 * nwg_line;
    if (groups > 2147483647LL) return hipErrorInvalidValue;
    const dim3 gr((unsigned)groups), b(256);
    switch (W) {
        case 1: hipLaunchKernelGGL(axis0_rotate_kernel<1>, gr, b, 0, s, T2, NL, ncp, m.n0, P, E, Ukq, nW, nm, nwg_line, g); break;
        case 3: hipLaunchKernelGGL(axis0_rotate_kernel<3>, gr, b, 0, s, T2, NL, ncp, m.n0, P, E, Ukq, nW, nm, nwg_line, g); break;
        case 5: hipLaunchKernelGGL(axis0_rotate_kernel<5>, gr, b, 0, s, T2, NL, ncp, m.n0, P, E, Ukq, nW, nm, nwg_line, g); break;
        default: hipLaunchKernelGGL(axis0_rotate_kernel<7>, gr, b, 0, s, T2, NL, ncp, m.n0, P, E, Ukq, nW, nm, nwg_line, g); break;
    }
    return hipGetLastError();
}

bool axis_transforms_fused(int rmax, int nc_pad, bool f32) {
    const int W = 2 * rmax + 1;
    const bool listed = W == 1 || W == 3 || W == 5 || W == 7 || W == 9;  // compile-time widths
    return listed && (size_t)W * W * 64 * (f32 ? sizeof(cf) : sizeof(cd)) <= 64 * 1024 &&
           nc_pad % 64 == 0;
}

hipError_t launch_axis_transforms(const cd* F, int rp_pad, int nc_pad, const int32_t* box_rp,
                                  int rmax, Mesh m, const cd* P, int nst, const uint32_t* line_any,
                                  cd* T1, cd* T2, hipStream_t s) {
    return axis_transforms<cd>(F, rp_pad, nc_pad, box_rp, rmax, m, P, nst, line_any, T1, T2, s);
}
hipError_t launch_axis_transforms_f32(const cf* F, int rp_pad, int nc_pad, const int32_t* box_rp,
                                      int rmax, Mesh m, const cd* P, int nst,
                                      const uint32_t* line_any, cf* T1, cf* T2, hipStream_t s) {
    return axis_transforms<cf>(F, rp_pad, nc_pad, box_rp, rmax, m, P, nst, line_any, T1, T2, s);
}

// ---------------------------------------------------------------------------
// Stage 1 (sum over Re at the kept k of a batch), factorised the same way.
// The kept k are mesh points, so e^{i2pi k.Re} = P0[k0, R0] P1[k1, R1]
// P2[k2, R2]; with Re embedded in its box (box_re: box position -> row of
// g(Re, Rp), -1 where the list has no vector) the sum is taken one axis at a
// time over the distinct k0 of the batch, then the distinct (k0, k1) pairs,
// then each k:
//   T0[d, R1 R2, c] = sum_R0 P0[k0_d, R0] g[R0 R1 R2, c]          (streams g once)
//   T1[p, R2, c]    = sum_R1 P1[k1_p, R1] T0[d(p), R1 R2, c]      (registers only)
//   G[row, c]       = sum_R2 P2[k2, R2] T1[p(row), R2, c]
// with c over the n_rp nModes nW^2 columns of g; C = cd, or cf for the FP32
// form (g rounded to FP32 as it is read).
// ---------------------------------------------------------------------------
template <int WT, class C>
__global__ __launch_bounds__(256) void re_axis0_kernel(const cd* __restrict__ g, int64_t NC,
                                                       const int32_t* __restrict__ box_re, int Wr,
                                                       const cd* __restrict__ P0,
                                                       const int32_t* __restrict__ d_k0, int d0,
                                                       int tr, C* __restrict__ T0) {
    constexpr int NV = WT > 0 ? WT : kMaxW;
    const int W = WT > 0 ? WT : Wr;
    const int64_t W2 = (int64_t)W * W;
    const int64_t total = W2 * NC;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = t % NC;
        const int64_t p = t / NC;
        // tr: every 16 x 16 (a, b) block of a column group is stored transposed,
        // T0 column (b, a) taking g column (a, b)
        const int64_t cg = tr ? ((c & ~(int64_t)255) | ((c & 15) << 4) | ((c >> 4) & 15)) : c;
        C v[NV];
#pragma unroll
        for (int r = 0; r < NV; ++r)
            if (r < W) {
                const int row = box_re[r * W2 + p];
                v[r] = row >= 0 ? to_c<C>(g[(int64_t)row * NC + cg]) : C{0, 0};
            }
        for (int d = 0; d < d0; ++d) {
            const cd* Pk = P0 + (int64_t)d_k0[d] * W;
            C acc = {0, 0};
#pragma unroll
            for (int r = 0; r < NV; ++r)
                if (r < W) acc = cfma(to_c<C>(Pk[r]), v[r], acc);
            T0[((int64_t)d * W2 + p) * NC + c] = acc;
        }
    }
}

// The (k0, k1) and k steps, fused: a work-group takes one distinct k0 (d) and
// 64 columns; T0[d, :, cols] (W^2 x 64) is staged in LDS once, and the four
// thread groups take the pairs of d in turn, each forming
//   T1[R2] = sum_R1 P1[k1, R1] T0[R1 R2]   in registers, then
//   G[row] = sum_R2 P2[k2, R2] T1[R2]      for the pair's rows,
// so the pair intermediate never reaches memory.
template <int WT, class C>
__global__ __launch_bounds__(256) void re_axis12_kernel(const C* __restrict__ T0, int64_t NC, int Wr,
                                                        const cd* __restrict__ P1,
                                                        const cd* __restrict__ P2,
                                                        const int32_t* __restrict__ pair_k1,
                                                        const int32_t* __restrict__ pair_off,
                                                        const int32_t* __restrict__ kp_off,
                                                        const int32_t* __restrict__ k_row,
                                                        const int32_t* __restrict__ k_k2,
                                                        const int32_t* __restrict__ d_plane,
                                                        int64_t ncb, C* __restrict__ G, int64_t ldg) {
    constexpr int NV = WT > 0 ? WT : kMaxW;
    const int W = WT > 0 ? WT : Wr;
    extern __shared__ char smem_raw[];
    C* sT = reinterpret_cast<C*>(smem_raw);  // [W^2][64]
    const int d = (int)(blockIdx.x / ncb);
    const int64_t c0 = (blockIdx.x % ncb) * 64;
    const int tid = threadIdx.x;
    // T0 plane of the batch's d-th distinct k0 (all planes resident, or the batch's own)
    const int plane = d_plane ? d_plane[d] : d;
    const C* src = T0 + (int64_t)plane * W * W * NC + c0;
    for (int i = tid; i < W * W * 64; i += 256) {
        const int rr = i >> 6, cc = i & 63;
        sT[i] = c0 + cc < NC ? src[(int64_t)rr * NC + cc] : C{0, 0};
    }
    __syncthreads();
    // the wave index is uniform across the wave: with it the pair and row
    // indices, and the phase-table reads they address, become scalar loads
    const int cc = tid & 63, tg = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t c = c0 + cc;
    // two pairs per pass (pp and pp + 4): every T0 value read from LDS feeds
    // two complex multiply-adds
    const int pend = pair_off[d + 1];
    for (int pp = pair_off[d] + tg; pp < pend; pp += 8) {
        const bool two = pp + 4 < pend;
        const cd* Pka = P1 + (int64_t)pair_k1[pp] * W;
        const cd* Pkb = P1 + (int64_t)pair_k1[two ? pp + 4 : pp] * W;
        C ta[NV], tb[NV];
#pragma unroll
        for (int r2 = 0; r2 < NV; ++r2) ta[r2] = tb[r2] = C{0, 0};
        // one R1 row at a time keeps the register footprint to the 2 W sums
        if (two) {  // (wave-uniform)
#pragma unroll 1
            for (int r1 = 0; r1 < W; ++r1) {
                const C pa = to_c<C>(Pka[r1]), pb = to_c<C>(Pkb[r1]);
                const C* row = sT + r1 * W * 64 + cc;
#pragma unroll
                for (int r2 = 0; r2 < NV; ++r2)
                    if (r2 < W) {
                        const C v = row[r2 * 64];
                        ta[r2] = cfma(pa, v, ta[r2]);
                        tb[r2] = cfma(pb, v, tb[r2]);
                    }
            }
        } else {  // the wave's last pair alone: no second set of products
#pragma unroll 1
            for (int r1 = 0; r1 < W; ++r1) {
                const C pa = to_c<C>(Pka[r1]);
                const C* row = sT + r1 * W * 64 + cc;
#pragma unroll
                for (int r2 = 0; r2 < NV; ++r2)
                    if (r2 < W) ta[r2] = cfma(pa, row[r2 * 64], ta[r2]);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && !two) break;
            const int p = pp + 4 * h;
            for (int i = kp_off[p]; i < kp_off[p + 1]; ++i) {
                const cd* Pk2 = P2 + (int64_t)k_k2[i] * W;
                C acc = {0, 0};
#pragma unroll
                for (int r2 = 0; r2 < NV; ++r2)
                    if (r2 < W) acc = cfma(to_c<C>(Pk2[r2]), h ? tb[r2] : ta[r2], acc);
                if (c < NC) G[(int64_t)k_row[i] * ldg + c] = acc;
            }
        }
    }
}

// Two 16-lane row sums at once by DPP: the first step (quad_perm 1,0,3,2) swaps
// the values so that each even lane adds the pair's a and each odd lane the pair's
// b; then quad_perm 2,3,0,1 and row rotations by 4 and by 8 add lanes of the same
// parity.  Every even lane of the row ends with the sum of a, every odd lane with
// the sum of b: half the moves and adds of two separate row sums.
// Every lane of the row reads a lane of the same row for these controls, so the
// moves take no old value (no zeroing instructions before them).
template <int CTRL>
__device__ inline double dpp_f64(double x) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int CTRL>
__device__ inline float dpp_f32(float x) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, true));
}
template <class R>
__device__ inline R row16_sum2(R a, R b, bool odd) {
    const R keep = odd ? b : a, send = odd ? a : b;
    R x;
    if constexpr (sizeof(R) == 8) {
        x = keep + dpp_f64<0xB1>(send);
        x += dpp_f64<0x4E>(x);
        x += dpp_f64<0x124>(x);
        x += dpp_f64<0x128>(x);
    } else {
        x = keep + dpp_f32<0xB1>(send);
        x += dpp_f32<0x4E>(x);
        x += dpp_f32<0x124>(x);
        x += dpp_f32<0x128>(x);
    }
    return x;
}

// The pair and k steps with the U_k fold of the rates applied at once (nW = 16):
// T0 holds every 16 x 16 (a, b) block transposed, so a 64-column block is
// (b = 4 qb + g, a = i) for lane (g, i) of each wave and
//   F[st, Rp, sa*16 + b] = sum_a conj(U_k[a, n_st]) G[k, Rp, sa, a, b]
// is a sum over the 16 lanes of a row.  G never leaves the registers; F is
// written once per state.
constexpr int kFoldWaves = 8;  // waves of the folded pair kernel sharing one T0 slab
// Waves per SIMD the folded pair kernel is compiled for: with a box of at most 7
// its FP64 slab (49 x 64 x 16 B) lets three work-groups share a CU, which needs
// six waves per SIMD (80 VGPRs); wider boxes fit one work-group per CU anyway.
template <int WT>
constexpr int fold_waves_per_simd() {
    return WT > 0 && WT <= 7 ? 6 : 2;
}

template <int WT, class C>
__global__ __launch_bounds__(64 * kFoldWaves, fold_waves_per_simd<WT>()) void re_axis12_fold_kernel(
    const C* __restrict__ T0, int64_t NC, int Wr, const cd* __restrict__ P1,
    const cd* __restrict__ P2, const int32_t* __restrict__ pair_k1,
    const int32_t* __restrict__ pair_off, const int32_t* __restrict__ kp_off,
    const int32_t* __restrict__ k_row, const int32_t* __restrict__ k_k2,
    const int32_t* __restrict__ d_plane, const int4* __restrict__ k_ent, int64_t ncb,
    FoldOut fo) {
    using R = decltype(C::x);
    constexpr int NV = WT > 0 ? WT : kMaxW;
    const int W = WT > 0 ? WT : Wr;
    extern __shared__ char smem_raw[];
    C* sT = reinterpret_cast<C*>(smem_raw);  // [W^2][64]
    const int d = (int)(blockIdx.x / ncb);
    const int64_t cb = blockIdx.x % ncb;
    const int64_t c0 = cb * 64;
    const int tid = threadIdx.x;
    const int plane = d_plane ? d_plane[d] : d;
    const C* src = T0 + (int64_t)plane * W * W * NC + c0;
    for (int i = tid; i < W * W * 64; i += 64 * kFoldWaves)
        st_vec(sT + i, ld_vec(src + (int64_t)(i >> 6) * NC + (i & 63)));
    __syncthreads();
    const int cc = tid & 63, tg = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = cc & 15, lg = cc >> 4;
    // column block -> (Rp row r, mode sa, b quarter)
    const int64_t grp = cb >> 2;
    const int r = (int)(grp / fo.nm), sa = (int)(grp - (int64_t)r * fo.nm);
    const int b = 4 * (int)(cb & 3) + lg;
    C* Fo = reinterpret_cast<C*>(fo.F) + (int64_t)r * fo.nc_pad + sa * 16 + b;
    const int64_t fst = (int64_t)fo.rp_pad * fo.nc_pad;
    const int pend = pair_off[d + 1];
    for (int pp = pair_off[d] + tg; pp < pend; pp += 2 * kFoldWaves) {
        const bool two = pp + kFoldWaves < pend;
        const cd* Pka = P1 + (int64_t)pair_k1[pp] * W;
        const cd* Pkb = P1 + (int64_t)pair_k1[two ? pp + kFoldWaves : pp] * W;
        C ta[NV], tb[NV];
#pragma unroll
        for (int r2 = 0; r2 < NV; ++r2) ta[r2] = tb[r2] = C{0, 0};
        if (two) {  // (wave-uniform) both pairs from one read of each slab value
#pragma unroll 1
            for (int r1 = 0; r1 < W; ++r1) {
                const C pa = to_c<C>(Pka[r1]), pbv = to_c<C>(Pkb[r1]);
                const C* row = sT + r1 * W * 64 + cc;
#pragma unroll
                for (int r2 = 0; r2 < NV; ++r2)
                    if (r2 < W) {
                        const C v = ld_vec(row + r2 * 64);
                        ta[r2] = cfma(pa, v, ta[r2]);
                        tb[r2] = cfma(pbv, v, tb[r2]);
                    }
            }
        } else {  // the wave's last pair alone: no second set of products
#pragma unroll 1
            for (int r1 = 0; r1 < W; ++r1) {
                const C pa = to_c<C>(Pka[r1]);
                const C* row = sT + r1 * W * 64 + cc;
#pragma unroll
                for (int r2 = 0; r2 < NV; ++r2)
                    if (r2 < W) ta[r2] = cfma(pa, ld_vec(row + r2 * 64), ta[r2]);
            }
        }
        // this lane's G[k, Rp r, sa, a = li, b], folded into every state of row k:
        // F = sum over the 16 lanes of the row of conj(U_k[a, n]) G
        auto fold = [&](const C& acc, int st) {
            const C u =
                to_c<C>(fo.U[((int64_t)fo.st_kmesh[st] * 16 + fo.st_band[st]) * 16 + li]);
            const R f = row16_sum2(u.x * acc.x + u.y * acc.y, u.x * acc.y - u.y * acc.x, li & 1);
            if (li < 2) reinterpret_cast<R*>(Fo + st * fst)[li] = f;  // Re from lane 0, Im from 1
        };
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && !two) break;
            const int p = pp + kFoldWaves * h;
            const int iend = kp_off[p + 1];
            // two k of the pair at a time: one record each (k2, first state, end of its
            // states), so their loads are issued together and the chains overlap
            for (int i = kp_off[p]; i < iend; i += 2) {
                const bool second = i + 1 < iend;
                const int4 ea = k_ent[i];
                const int4 eb = k_ent[second ? i + 1 : i];
                const cd* Pa = P2 + (int64_t)ea.x * W;
                const cd* Pb = P2 + (int64_t)eb.x * W;
                C aa = {0, 0}, ab = {0, 0};
#pragma unroll
                for (int r2 = 0; r2 < NV; ++r2)
                    if (r2 < W) {
                        const C t = h ? tb[r2] : ta[r2];
                        aa = cfma(to_c<C>(Pa[r2]), t, aa);
                        ab = cfma(to_c<C>(Pb[r2]), t, ab);
                    }
                for (int st = ea.y; st < ea.z; ++st) fold(aa, st);
                if (second)
                    for (int st = eb.y; st < eb.z; ++st) fold(ab, st);
            }
        }
    }
}

template <int WT, class C>
static hipError_t go_re_axis0(const cd* g, int64_t NC, const int32_t* box_re, int W, const cd* P,
                              const int32_t* k0_list, int n, bool tr, C* T0, hipStream_t s) {
    hipLaunchKernelGGL((re_axis0_kernel<WT, C>), dim3(gridm((int64_t)W * W * NC, 256)), dim3(256),
                       0, s, g, NC, box_re, W, P, k0_list, n, tr ? 1 : 0, T0);
    return hipGetLastError();
}

template <int WT, class C>
static hipError_t go_re_axis12(const C* T0, int64_t NC, int W, Mesh m, const cd* P,
                               const ReBatch& b, const FoldOut* fo, C* G, int64_t ldg,
                               hipStream_t s) {
    const cd* P1 = P + (int64_t)m.n0 * W;
    const cd* P2 = P1 + (int64_t)m.n1 * W;
    const size_t shm = (size_t)W * W * 64 * sizeof(C);
    const void* kern = fo ? (const void*)re_axis12_fold_kernel<WT, C>
                          : (const void*)re_axis12_kernel<WT, C>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    const int64_t ncb = (NC + 63) / 64;
    if ((int64_t)b.d0 * ncb > 2147483647LL) return hipErrorInvalidValue;
    if (fo && (!b.k_ent || (reinterpret_cast<uintptr_t>(b.k_ent) & 15))) return hipErrorInvalidValue;
    if (fo)
        hipLaunchKernelGGL((re_axis12_fold_kernel<WT, C>), dim3((unsigned)(b.d0 * ncb)),
                           dim3(64 * kFoldWaves),
                           shm, s, T0, NC, W, P1, P2, b.pair_k1, b.pair_off, b.kp_off, b.k_row,
                           b.k_k2, b.d_plane, reinterpret_cast<const int4*>(b.k_ent), ncb, *fo);
    else
        hipLaunchKernelGGL((re_axis12_kernel<WT, C>), dim3((unsigned)(b.d0 * ncb)), dim3(256), shm,
                           s, T0, NC, W, P1, P2, b.pair_k1, b.pair_off, b.kp_off, b.k_row, b.k_k2,
                           b.d_plane, ncb, G, ldg);
    return hipGetLastError();
}

// the folded form needs nW = 16 (a 64-column block is 4 b x 16 a of one Rp row
// and mode) and F columns sa*16 + b
static bool fold_ok(const FoldOut* fo, int64_t NC) {
    return !fo || (fo->nW == 16 && NC == (int64_t)fo->n_rp * fo->nm * 256 && fo->nc_pad >= 16 * fo->nm &&
                   fo->rp_pad >= fo->n_rp && fo->row_st && fo->st_kmesh && fo->st_band && fo->U &&
                   fo->F);
}

// the box width as a compile-time constant where it is a common one
template <class F>
static hipError_t with_box_width(int W, F&& f) {
    switch (W) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 5: return f(std::integral_constant<int, 5>{});
        case 7: return f(std::integral_constant<int, 7>{});
        case 9: return f(std::integral_constant<int, 9>{});
        default: return f(std::integral_constant<int, 0>{});
    }
}

// LDS of the fused kernel: W^2 x 64 staged values
size_t re_axes_lds(int rmax, bool f32) {
    const int W = 2 * rmax + 1;
    return (size_t)W * W * 64 * (f32 ? sizeof(cf) : sizeof(cd));
}

template <class C>
static hipError_t re_axes(const cd* g, int64_t NC, const int32_t* box_re, int rmax, Mesh m,
                          const cd* P, const ReBatch& b, const FoldOut* fo, C* T0, C* G,
                          int64_t ldg, hipStream_t s) {
    const int W = 2 * rmax + 1;
    if (W > kMaxW || b.d0 <= 0 || b.d01 <= 0 || b.d_plane || !fold_ok(fo, NC) ||
        re_axes_lds(rmax, sizeof(C) == sizeof(cf)) > 160 * 1024)
        return hipErrorInvalidValue;
    return with_box_width(W, [&](auto wt) {
        constexpr int WT = decltype(wt)::value;
        hipError_t e = go_re_axis0<WT, C>(g, NC, box_re, W, P, b.d_k0, b.d0, fo != nullptr, T0, s);
        if (e != hipSuccess) return e;
        return go_re_axis12<WT, C>(T0, NC, W, m, P, b, fo, G, ldg, s);
    });
}

template <class C>
static hipError_t re_planes(const cd* g, int64_t NC, const int32_t* box_re, int rmax,
                            const cd* P, const int32_t* k0_list, int n, bool tr, C* T0,
                            hipStream_t s) {
    const int W = 2 * rmax + 1;
    if (W > kMaxW || n <= 0 || (tr && NC % 256 != 0)) return hipErrorInvalidValue;
    return with_box_width(W, [&](auto wt) {
        return go_re_axis0<decltype(wt)::value, C>(g, NC, box_re, W, P, k0_list, n, tr, T0, s);
    });
}

template <class C>
static hipError_t re_pairs(const C* T0, int64_t NC, int rmax, Mesh m, const cd* P,
                           const ReBatch& b, const FoldOut* fo, C* G, int64_t ldg, hipStream_t s) {
    const int W = 2 * rmax + 1;
    if (W > kMaxW || b.d0 <= 0 || b.d01 <= 0 || !b.d_plane || !fold_ok(fo, NC) ||
        re_axes_lds(rmax, sizeof(C) == sizeof(cf)) > 160 * 1024)
        return hipErrorInvalidValue;
    return with_box_width(W, [&](auto wt) {
        return go_re_axis12<decltype(wt)::value, C>(T0, NC, W, m, P, b, fo, G, ldg, s);
    });
}

hipError_t launch_re_axes(const cd* g, int64_t NC, const int32_t* box_re, int rmax, Mesh m,
                          const cd* P, const ReBatch& b, const FoldOut* fo, cd* T0, cd* G,
                          int64_t ldg, hipStream_t s) {
    return re_axes<cd>(g, NC, box_re, rmax, m, P, b, fo, T0, G, ldg, s);
}
hipError_t launch_re_axes_f32(const cd* g, int64_t NC, const int32_t* box_re, int rmax, Mesh m,
                              const cd* P, const ReBatch& b, const FoldOut* fo, cf* T0, cf* G,
                              int64_t ldg, hipStream_t s) {
    return re_axes<cf>(g, NC, box_re, rmax, m, P, b, fo, T0, G, ldg, s);
}
hipError_t launch_re_planes(const cd* g, int64_t NC, const int32_t* box_re, int rmax,
                            const cd* P, const int32_t* k0_list, int n, bool tr, cd* T0,
                            hipStream_t s) {
    return re_planes<cd>(g, NC, box_re, rmax, P, k0_list, n, tr, T0, s);
}
hipError_t launch_re_planes_f32(const cd* g, int64_t NC, const int32_t* box_re, int rmax,
                                const cd* P, const int32_t* k0_list, int n, bool tr, cf* T0,
                                hipStream_t s) {
    return re_planes<cf>(g, NC, box_re, rmax, P, k0_list, n, tr, T0, s);
}
hipError_t launch_re_pairs(const cd* T0, int64_t NC, int rmax, Mesh m, const cd* P,
                           const ReBatch& b, const FoldOut* fo, cd* G, int64_t ldg, hipStream_t s) {
    return re_pairs<cd>(T0, NC, rmax, m, P, b, fo, G, ldg, s);
}
hipError_t launch_re_pairs_f32(const cf* T0, int64_t NC, int rmax, Mesh m, const cd* P,
                               const ReBatch& b, const FoldOut* fo, cf* G, int64_t ldg,
                               hipStream_t s) {
    return re_pairs<cf>(T0, NC, rmax, m, P, b, fo, G, ldg, s);
}

// ---------------------------------------------------------------------------
// Last axis on MFMA + rotations + rate terms.  Work-group = one state x one
// (q1, q2) line; its live points are taken 16 at a time.  The MFMA computes
// the transposed tile X^T[b, q0] = sum_R0 T2[R0, col b] P0[q0, R0]: lane l
// feeds A[l%16][l/16] = T2[R0, line, col] and B[l/16][l%16] = P0[q0, R0].
//
// Columns are laid out c = sa*16 + b (b < nW <= 16), so every 16-column tile
// holds one mode index sa.  The tile's rows are ordered so that lane (g, i)
// (g = l/16, i = l%16) ends up with X[q0 = i, sa, b = 4g + v] in its result
// register v (FP64 16x16x4: result row g + 4v, so row r loads column
// b = 4(r%4) + r/4; FP32 16x16x4: result row 4g + v, natural order).  The k+q
// rotation
//   Y[q, sa, m] = sum_b X[q, sa, b] U_{k+q}[b, m]
// is then four products per lane and a sum over the four 16-lane rows, done
// for four vectors at once with the gfx950 lane swaps.  Only Y (16 q x modes,
// one final band at a time) goes through LDS to the threads that apply
// E_q = z l and form the rate terms.
// ---------------------------------------------------------------------------
// permlane32_swap exchanges lanes 32-63 of a with lanes 0-31 of b;
// permlane16_swap exchanges the odd 16-lane rows of a with the even rows of b.
template <int ROWS>
__device__ inline void lane_swap(uint32_t& a, uint32_t& b) {
    if constexpr (ROWS == 2) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}
template <int ROWS>
__device__ inline void lane_swap(double& a, double& b) {
    const uint64_t x = __builtin_bit_cast(uint64_t, a), y = __builtin_bit_cast(uint64_t, b);
    uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32), yl = (uint32_t)y, yh = (uint32_t)(y >> 32);
    lane_swap<ROWS>(xl, yl);
    lane_swap<ROWS>(xh, yh);
    a = __builtin_bit_cast(double, ((uint64_t)xh << 32) | xl);
    b = __builtin_bit_cast(double, ((uint64_t)yh << 32) | yl);
}
template <int ROWS>
__device__ inline void lane_swap(float& a, float& b) {
    uint32_t x = __builtin_bit_cast(uint32_t, a), y = __builtin_bit_cast(uint32_t, b);
    lane_swap<ROWS>(x, y);
    a = __builtin_bit_cast(float, x);
    b = __builtin_bit_cast(float, y);
}

// Four sums over the four 16-lane rows at once: on return lane (g, i) holds
// sum_{g'} u_g[g', i], i.e. row 0 the sum of u0, row 1 of u1, row 2 of u2 and
// row 3 of u3.  After the 32-lane swap and add, lanes 0-31 hold half sums of
// u0 (u1) and lanes 32-63 of u2 (u3); the 16-lane swap and add completes them.
template <class R>
__device__ inline R rows4_reduce_scatter(R u0, R u1, R u2, R u3) {
    lane_swap<2>(u0, u2);
    lane_swap<2>(u1, u3);
    R s = u0 + u2, t = u1 + u3;
    lane_swap<4>(s, t);
    return s + t;
}

// Live final bands of every point.  Bit m of live[(st * NL + line) * N0 + q0]
// is set when |eps_n - eps_{m,k+q}| <= 27.5 sigma + max omega at that point;
// otherwise both Gaussians of every term of band m there are beyond 27.5 sigma,
// i.e. exactly 0.  One thread per (state, line), the line index fastest; the
// masks of one line are contiguous, so the line kernel reads them as one
// block.  The thread also leaves
// the union of its line's bands in line_bands and counts (one atomic per wave)
// n_live[0] the lines with a live band and n_live[1] the units of 16 points the
// line kernel will take (per band, its live points / 16 rounded up), and writes
// the zero partial sum of every pair without a live band.
__global__ __launch_bounds__(256, 8) void line_live_kernel(RateArgs a, uint32_t* __restrict__ live,
                                 uint32_t* __restrict__ line_bands, uint32_t* __restrict__ n_live) {
    const Mesh mesh = a.mesh;
    const int N0 = mesh.n0, NL = mesh.n1 * mesh.n2, nW = a.nW;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint32_t u = 0, units = 0;
    if (i < (int64_t)a.n_states * NL) {
        const int line = (int)(i % NL), st = (int)(i / NL);
        const int q1 = line / mesh.n2, q2 = line - q1 * mesh.n2;
        const int kmesh = a.st_kmesh[st];
        const int mlo = a.st_mlo[st], mhi = a.st_mhi[st];
        int k0i, k1i, k2i;
        mesh_triple(kmesh, mesh, k0i, k1i, k2i);
        const int64_t kq12 = ((k1i + q1) % mesh.n1) * mesh.n2 + (k2i + q2) % mesh.n2;
        const double eps_n = a.eps[(int64_t)kmesh * nW + a.st_band[st]];
        const double lim = 27.5 * a.sigma + *a.wmax;
        uint32_t cnt2[16] = {};  // live points per band, two 16-bit counts a word (N0 <= 1024)
        uint32_t* out = live + i * N0;
        // band values two at a time (16-byte loads from an even band; rows are
        // nW doubles, nW even here); masks four at a time where N0 % 4 == 0
        const bool pairs = (nW & 1) == 0;
        // adaptive smearing: each band's limit uses its own width at the point
        const double* vn = a.vel ? a.vel + ((int64_t)kmesh * nW + a.st_band[st]) * 3 : nullptr;
        auto bits_of = [&](int q0) {
            const int64_t kq = (int64_t)((k0i + q0) % N0) * NL + kq12;
            const double* ek = a.eps + kq * nW;
            uint32_t bits = 0;
            if (vn) {
                const double wm = *a.wmax;
                for (int m = mlo; m <= mhi; ++m) {
                    const double* vm = a.vel + (kq * nW + m) * 3;
                    double s2 = 0.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const double t = a.ad_c[d] * (vn[d] - vm[d]);
                        s2 += t * t;
                    }
                    const double sg = fmax(a.sigma, sqrt(s2));
                    bits |= (uint32_t)(fabs(eps_n - ek[m]) <= 27.5 * sg + wm) << m;
                }
            } else if (pairs) {
                for (int m = mlo & ~1; m <= mhi; m += 2) {
                    const double2 e2 = *reinterpret_cast<const double2*>(ek + m);
                    bits |= (uint32_t)(m >= mlo && fabs(eps_n - e2.x) <= lim) << m;
                    bits |= (uint32_t)(m + 1 <= mhi && fabs(eps_n - e2.y) <= lim) << (m + 1);
                }
            } else {
                for (int m = mlo; m <= mhi; ++m) bits |= (uint32_t)(fabs(eps_n - ek[m]) <= lim) << m;
            }
            u |= bits;
#pragma unroll
            for (int m = 0; m < 32; ++m) cnt2[m >> 1] += ((bits >> m) & 1u) << (16 * (m & 1));
            return bits;
        };
        if ((N0 & 3) == 0) {
            for (int q0 = 0; q0 < N0; q0 += 4) {
                uint4 v;
                v.x = bits_of(q0);
                v.y = bits_of(q0 + 1);
                v.z = bits_of(q0 + 2);
                v.w = bits_of(q0 + 3);
                *reinterpret_cast<uint4*>(out + q0) = v;
            }
        } else {
#pragma unroll 4
            for (int q0 = 0; q0 < N0; ++q0) out[q0] = bits_of(q0);
        }
        line_bands[i] = u;
        if (!u) a.partial[(int64_t)st * a.n_qtiles + line] = 0.0;  // the line kernel skips the pair
#pragma unroll
        for (int m = 0; m < 32; ++m) units += (((cnt2[m >> 1] >> (16 * (m & 1))) & 0xFFFFu) + 15) / 16;
    }
    const uint64_t bal = __ballot(u != 0);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) units += __shfl_xor(units, o, 64);
    if ((threadIdx.x & 63) == 0) {
        if (bal) atomicAdd(n_live, (uint32_t)__popcll(bal));
        if (units) atomicAdd(n_live + 1, units);
    }
}

hipError_t launch_line_live(const RateArgs& a, int nst, uint32_t* live, uint32_t* line_bands,
                            uint32_t* n_live, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    if (a.nW > 32 || !live || !line_bands || !n_live || !a.partial ||
        a.n_qtiles != a.mesh.n1 * a.mesh.n2)
        return hipErrorInvalidValue;
    RateArgs b = a;
    b.n_states = nst;
    const int64_t n = (int64_t)nst * a.mesh.n1 * a.mesh.n2;
    hipLaunchKernelGGL(line_live_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b, live,
                       line_bands, n_live);
    return hipGetLastError();
}

__device__ inline d4 mfma16(double x, double y, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}
__device__ inline f4 mfma16(float x, float y, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
}

// C = cd: FP64 on v_mfma_f64_16x16x4f64; C = cf: the FP32 form on
// v_mfma_f32_16x16x4f32, with the rotations in FP32 and the Gaussian terms and
// sums in FP64.
//
// A work-group takes the live final bands of its line in order; for each band
// it lists the band's live points (a wave ballot over the point masks) and
// works through the list 16 points at a time, so that every MFMA row and
// every term item belongs to a live point where possible.  The phase rows, the
// eigenvectors at k+q and the band and phonon values of a unit are gathered
// through the list; the last group of a band is padded with an all-zero
// phase row.  Only the E_q loads of the terms that survive the Gaussian test
// wait on memory after the rotation.
//
// KS > 0 (lines of at most 4 KS rows of T2): the work-group's T2 fragments are
// loaded into registers right after the live test, behind the point masks and
// the phase table, so that the three are in flight together and the list
// building and the unit's gathers overlap them; KS = 0 loads them per K step.
constexpr int kTP = 2;  // column tiles per MFMA pass

// FEAT (FP64 only, a bit set; 0 for the plain rates): kLineLW linewidth
// partials, kLinePol the polar term, kLineVel adaptive widths.  Each variant
// carries only the registers of its own terms.
// partials (RateArgs.Lpol / vel / lw), each switched on by its pointer.
// Waves per SIMD the line kernel is compiled for: four for the plain rates; the
// extension terms, and the FP64 form with two tiles per mode (its U_{k+q} values
// of both halves), need more registers, and at four waves they would spill.
constexpr int kLineLW = 1, kLinePol = 2, kLineVel = 4;
template <int FEAT, int H, bool F64, int NWV = 4>
constexpr int line_waves_per_simd() {
    if (NWV == 2) return FEAT & kLinePol ? 2 : 3;  // two waves per work-group: twice the tiles per wave
    if (H == 2 && F64) return FEAT == 0 || FEAT == kLineLW ? 3 : 2;
    return FEAT == 0 || FEAT == kLineLW ? 4 : 3;
}

// H: column tiles per mode, 1 (nW <= 16: column sa*16 + b) or 2 (nW <= 32: column
// sa*32 + b, the tiles of a mode being its halves b < 16 and b >= 16, one MFMA pass).
// NWV: waves per work-group, 4, or 2 with twice the tiles per wave: a pair then
// holds 2 x 159 VGPRs per lane instead of 4 x 127, so six (state, line) pairs are
// resident per CU instead of four (measured on the realistic workload: 2.45 ms per
// launch against 2.68 ms; one wave of sixteen tiles, 2.47 ms; two waves loading
// T2 per K step, 2.73 ms).  The plain rates of two and three tiles per wave take the
// two-wave form as well (the batched plan of 32 systems: 137.9 -> 133.9 ms), and so do
// the linewidth and adaptive-width variants (163 VGPRs; phonon linewidth 107 -> 101.5 ms,
// adaptive rates 541 -> 478 ms per step) and, at two waves per SIMD (181 VGPRs; four
// pairs per CU against three), the polar one (3.29 -> 3.16 ms per launch); with two
// tiles per mode (16 < nW <= 32) the plain rates of one and two modes per wave, the
// latter in FP32 (batched plan 133.4 -> 132.1 ms); and the plain rates of six and eight
// tiles per wave, whose T2 is read per K step (12 and 16 tiles in two waves: 132.1 ->
// 129.9 ms), with one or two tiles per mode (-> 128.6 ms).
template <int TN, int KS, class C, int FEAT, int H = 1, int NWV = 4>
__global__ __launch_bounds__(64 * NWV, (line_waves_per_simd<FEAT, H, sizeof(C) == sizeof(cd), NWV>())) void
line_rates_kernel(RateArgs a) {
    constexpr int BT = 64 * NWV;  // threads of the work-group
    static_assert(H == 1 || (H == 2 && TN % 2 == 0 && kTP == 2),
                  "two tiles per mode: whole modes per wave and per pass");
    constexpr bool LW = FEAT & kLineLW, POL = FEAT & kLinePol, VEL = FEAT & kLineVel;
    using R = decltype(C::x);
    constexpr bool F64 = sizeof(R) == 8;
    using V4 = std::conditional_t<F64, d4, f4>;
    extern __shared__ char smem_raw[];
    const int W = a.W;
    const int Wp = (W + 3) & ~3;
    const int nW = a.nW, nm = a.nm;
    const Mesh mesh = a.mesh;
    const int N0 = mesh.n0;
    const int ldf = a.nc_pad;
    // phase table rows are Wp + 1 elements apart: the 16 rows an MFMA step reads then
    // start on different LDS banks (Wp apart, every other row would share banks)
    const int Ws = Wp + 1;
    C* sP = reinterpret_cast<C*>(smem_raw);                    // [N0 + 1][Ws], row N0 zero
    C* sY = sP + (N0 + 1) * Ws;                                // [16][nm]
    uint32_t* sPm = reinterpret_cast<uint32_t*>(sY + 16 * nm);  // [N0] live bands per point
    int* sList = reinterpret_cast<int*>(sPm + N0);             // [N0] live points of a band
    // LW: [N0][nm] linewidth partials of the work-group (8-byte aligned: N0 ints above)
    double* sLW = reinterpret_cast<double*>(sList + N0 + (N0 & 1));
    __shared__ double sRed[NWV];
    __shared__ int sCount;
    __shared__ cd sO[16];  // POL: overlap [U_k^dagger U_{k+q}]_{n m} at the unit's points

    // XCD-aware order: work-groups are dealt to the 8 XCDs round-robin, so
    // with id = 8 j + x every state of a line lands on XCD x, one after
    // another, and the line's phonon tables E_q are fetched into one L2 once.
    const int NL = mesh.n1 * mesh.n2;
    const int nst = a.n_states;
    const int64_t id = blockIdx.x;
    const int xcd = (int)(id & 7);
    const int64_t j = id >> 3;
    const int line = (int)((j / nst) * 8 + xcd);
    const int st = (int)(j % nst);
    if (line >= NL) return;
    uint32_t bands = a.line_bands[(int64_t)st * NL + line];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (!bands) return;  // its partial sum is 0 (written with the masks)
    const int q1 = line / mesh.n2, q2 = line - q1 * mesh.n2;
    const int li = lane & 15, lg = lane >> 4;
    const int kmesh = a.st_kmesh[st];
    const int nband = a.st_band[st];
    int k0i, k1i, k2i;
    mesh_triple(kmesh, mesh, k0i, k1i, k2i);
    const int kq12 = ((k1i + q1) % mesh.n1) * mesh.n2 + (k2i + q2) % mesh.n2;
    const int q12 = q1 * mesh.n2 + q2;
    const double eps_n = a.eps[(int64_t)kmesh * nW + nband];
    const double inv_s2 = 1.0 / (a.sigma * a.sigma);
    // |y| > 27.5 sigma: y^2/sigma^2 > 756 and exp(-756) is below the smallest
    // FP64 subnormal, so such a Gaussian is exactly 0
    const double cut = 27.5 * a.sigma;
    // per-state values of the extensions: U_k column n (lane rows 4 lg + v), v_nk, f (1 - f) / kT
    cd ukn[4 * H] = {};
    double vn[3] = {0.0, 0.0, 0.0};
    double mdf = 0.0;
    if constexpr (POL || VEL || LW) {
        if (POL && a.Lpol) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
                for (int h = 0; h < H; ++h)
                    if (16 * h + 4 * lg + v < nW)
                        ukn[4 * h + v] = a.U[((int64_t)kmesh * nW + nband) * nW + 16 * h + 4 * lg + v];
        }
        if (VEL && a.vel)
            for (int d = 0; d < 3; ++d) vn[d] = a.vel[((int64_t)kmesh * nW + nband) * 3 + d];
        if (LW && a.lw) {
            const double fn = a.focc[(int64_t)kmesh * nW + nband];
            mdf = fn * (1.0 - fn) * a.inv_kT;
            for (int i = tid; i < N0 * nm; i += BT) sLW[i] = 0.0;
        }
    }
    // tile row li loads column b = perm(li), see above
    const int bcol = F64 ? (((li & 3) << 2) | (li >> 2)) : li;
    const C* Tst = reinterpret_cast<const C*>(a.T2) + (int64_t)st * W * NL * ldf +
                   (int64_t)line * ldf + wave * TN * 16 + bcol;
    const int64_t Tk = (int64_t)NL * ldf;  // stride of R0 in T2

    const uint32_t* lv = a.live + ((int64_t)st * NL + line) * N0;
    const int nP = (N0 + 1) * Ws;
    auto p0_at = [&](int i) {
        const int q0 = i / Ws, r = i - q0 * Ws;
        return (q0 < N0 && r < W) ? to_c<C>(a.P0[q0 * W + r]) : C{0, 0};
    };
    // The first mask and table elements and the T2 fragments are loaded
    // without branches (clamped addresses), so that the LDS stores wait on
    // the first two only and T2 stays in flight.  A T2 row k >= W is read
    // from row W - 1 and meets a zero phase (the table is zero beyond W).
    const int i0 = min(tid, nP - 1), i1 = min(tid + BT, nP - 1);
    auto p0_src = [&](int i) {
        const int q0 = i / Ws, r = i - q0 * Ws;
        return a.P0[min(q0, N0 - 1) * W + min(r, W - 1)];
    };
    const uint32_t pm0 = lv[min(tid, N0 - 1)];
    const cd pv0 = p0_src(i0), pv1 = p0_src(i1);
    __builtin_amdgcn_sched_barrier(0);  // keep the T2 loads behind these
    C tb[KS > 0 ? KS * TN : 1];
    if constexpr (KS > 0) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int64_t k = min(4 * ks + lg, W - 1);
#pragma unroll
            for (int t = 0; t < TN; ++t) tb[ks * TN + t] = Tst[k * Tk + t * 16];
        }
    }
    auto p0_keep = [&](int i) {
        const int q0 = i / Ws, r = i - q0 * Ws;
        return q0 < N0 && r < W;
    };
    if (tid < N0) sPm[tid] = pm0;
    if (tid < nP) sP[tid] = p0_keep(tid) ? to_c<C>(pv0) : C{0, 0};
    if (tid + BT < nP) sP[tid + BT] = p0_keep(tid + BT) ? to_c<C>(pv1) : C{0, 0};
    for (int q0 = tid + BT; q0 < N0; q0 += BT) sPm[q0] = lv[q0];
    for (int i = tid + 2 * BT; i < nP; i += BT) sP[i] = p0_at(i);

    // Values one unit (band m, points list[g .. g+15]) needs: per lane,
    // U_{k+q}[b = 4 lg + v, m] at the lane's point; per thread, for its term
    // item (point slot c = tid / nm, mode nu = tid % nm), eps and f of band m
    // at k+q and omega and n of (q, nu).  Items beyond the first of a thread
    // (nm > 16) read theirs in place.
    struct Unit {
        C u[4 * H];  // U_{k+q}[b, m] at b = 16 h + 4 lg + v, entry 4 h + v
        double em, fm, om, nbq;
    };
    const bool has_item = tid < 16 * nm;
    const int ic = tid / nm, inu = tid - ic * nm;
    auto kq_of = [&](int q0) { return (int64_t)((k0i + q0) % N0) * NL + kq12; };
    auto load_unit = [&](int pl, int pc, int m, Unit& d) {
        // pl: this lane's point (-1: padding); pc: this thread's item point
        const int64_t kql = pl >= 0 ? kq_of(pl) : 0;
        const cd* Ur = a.U + (kql * nW + m) * nW + 4 * lg;
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                d.u[4 * h + v] =
                    (pl >= 0 && 16 * h + 4 * lg + v < nW) ? to_c<C>(Ur[16 * h + v]) : C{0, 0};
        d.em = d.fm = d.om = d.nbq = 0.0;
        if (has_item && pc >= 0) {
            const int64_t q = (int64_t)pc * NL + q12;
            const int64_t kq = kq_of(pc);
            d.em = a.eps[kq * nW + m];
            d.fm = a.focc[kq * nW + m];
            d.om = a.omega[q * nm + inu];
            d.nbq = a.nb[q * nm + inu];
        }
    };
    // rate term of one item; E_q is read only for terms that survive the test
    double gacc = 0.0;
    auto item_term = [&](int q0, int c, int nu, double em, double fm, double w, double nbq, int m) {
        const double x = eps_n - em;
        const double y1 = x - w, y2 = x + w;
        double is2 = inv_s2, cutv = cut, wt = 1.0;
        if constexpr (VEL) {
            if (a.vel) {  // adaptive width of the transition (k n) -> (k+q m)
                const double* vm = a.vel + (kq_of(q0) * nW + m) * 3;
                double s2 = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double t = a.ad_c[d] * (vn[d] - vm[d]);
                    s2 += t * t;
                }
                const double sg = fmax(a.sigma, sqrt(s2));
                is2 = 1.0 / (sg * sg);
                cutv = 27.5 * sg;
                wt = 1.0 / sg;
            }
        }
        // both Gaussians underflow to exactly 0: the term is 0
        if (fabs(y1) > cutv && fabs(y2) > cutv) return;
        const int64_t q = (int64_t)q0 * NL + q12;
        const C* Yr = sY + c * nm;
        const cd* Eq = a.E + (q * nm + nu) * nm;
        C z = {0, 0};
        for (int sa = 0; sa < nm; ++sa) z = cfma(to_c<C>(Eq[sa]), Yr[sa], z);
        if constexpr (POL) {
            if (a.Lpol) {  // + i L(q, nu) O_nm
                const cd l = a.Lpol[q * nm + nu];
                const cd o = sO[c];
                z.x -= l.x * o.y + l.y * o.x;
                z.y += l.x * o.x - l.y * o.y;
            }
        }
        const double g1 = wt * exp(-y1 * y1 * is2), g2 = wt * exp(-y2 * y2 * is2);
        const double z2 = cabs2(z);
        const double term = z2 * ((nbq + 1.0 - fm) * g1 + (nbq + fm) * g2);
        gacc += term;
        if (a.terms)
            atomicAdd(&a.terms[((int64_t)st * a.nq_mesh + q) * nm + nu], a.terms_scale * term);
        if constexpr (LW) {
            if (a.lw) sLW[q0 * nm + nu] += mdf * z2 * g1;  // one thread per (q0, nu) per unit
        }
    };

    __syncthreads();  // sPm, sP
    while (bands) {
        const int m = __builtin_ctz(bands);
        bands &= bands - 1;
        // live points of band m, ascending
        if (wave == 0) {
            int base = 0;
            for (int w0 = 0; w0 < N0; w0 += 64) {
                const int p = w0 + lane;
                const bool bit = p < N0 && ((sPm[p] >> m) & 1u);
                const uint64_t bal = __ballot(bit);
                if (bit) sList[base + __popcll(bal & ((1ull << lane) - 1ull))] = p;
                base += __popcll(bal);
            }
            if (lane == 0) sCount = base;
        }
        __syncthreads();
        const int cnt = sCount;
        if (cnt == 0) __syncthreads();  // (a band of the union has a point; kept for safety)
        for (int g = 0; g < cnt; g += 16) {
            const int pl = g + li < cnt ? sList[g + li] : -1;
            const int pc = has_item && g + ic < cnt ? sList[g + ic] : -1;
            Unit d;
            load_unit(pl, pc, m, d);
            const int prow = (pl >= 0 ? pl : N0) * Ws;
            // X^T tiles of the unit's points and Y, two column tiles at a time
#pragma unroll
            for (int t0 = 0; t0 < TN; t0 += kTP) {
                constexpr int P = TN < kTP ? TN : kTP;
                V4 cr[P], ci[P];
#pragma unroll
                for (int t = 0; t < P; ++t) {
                    cr[t] = V4{0, 0, 0, 0};
                    ci[t] = V4{0, 0, 0, 0};
                }
                auto kstep = [&](const C (&bc)[P], const C ph) {
#pragma unroll
                    for (int t = 0; t < P; ++t) {
                        cr[t] = mfma16(bc[t].x, ph.x, cr[t]);
                        ci[t] = mfma16(bc[t].y, ph.x, ci[t]);
                    }
#pragma unroll
                    for (int t = 0; t < P; ++t) {
                        cr[t] = mfma16(bc[t].y, -ph.y, cr[t]);
                        ci[t] = mfma16(bc[t].x, ph.y, ci[t]);
                    }
                };
                if constexpr (KS > 0) {
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        if (4 * ks >= Wp) break;
                        C bc[P];
#pragma unroll
                        for (int t = 0; t < P; ++t) bc[t] = t0 + t < TN ? tb[ks * TN + t0 + t] : C{0, 0};
                        kstep(bc, ld_vec(sP + prow + 4 * ks + lg));
                    }
                } else {
                    for (int k0 = 0; k0 < Wp; k0 += 4) {
                        const int k = k0 + lg;
                        C bc[P];
#pragma unroll
                        for (int t = 0; t < P; ++t)
                            bc[t] = (k < W && t0 + t < TN) ? Tst[k * Tk + (t0 + t) * 16] : C{0, 0};
                        kstep(bc, ld_vec(sP + prow + k));
                    }
                }
                // Y[slot li, sa] = sum_b X[slot li, sa, b] U_{k+q}[b, m]: products over
                // the lane's four b, then the sum over the four rows; rows 0/1 receive
                // Re Y of tiles t/t+1, rows 2/3 Im Y of tiles t/t+1.
                R pr[P], pi[P];
#pragma unroll
                for (int t = 0; t < P; ++t) {
                    const C* uu = d.u + (H == 2 ? 4 * t : 0);  // H = 2: tile t is half t
                    R xr = 0, xi = 0;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        xr += cr[t][v] * uu[v].x - ci[t][v] * uu[v].y;
                        xi += cr[t][v] * uu[v].y + ci[t][v] * uu[v].x;
                    }
                    pr[t] = xr;
                    pi[t] = xi;
                }
                if constexpr (H == 1) {
#pragma unroll
                    for (int t = 0; t < P; t += 2) {
                        const R y = rows4_reduce_scatter(pr[t], t + 1 < P ? pr[t + 1] : R(0), pi[t],
                                                         t + 1 < P ? pi[t + 1] : R(0));
                        const int tt = t0 + t + (lg & 1);
                        const int sa = wave * TN + tt;
                        if (t + (lg & 1) < P && tt < TN && sa < nm)
                            reinterpret_cast<R*>(sY + li * nm + sa)[lg >> 1] = y;
                    }
                } else {
                    // both halves of mode sa: Y is their sum; rows 0 and 2 receive Re and Im
                    const R y = rows4_reduce_scatter(pr[0] + pr[1], R(0), pi[0] + pi[1], R(0));
                    const int sa = (wave * TN + t0) >> 1;
                    if (!(lg & 1) && sa < nm) reinterpret_cast<R*>(sY + li * nm + sa)[lg >> 1] = y;
                }
            }
            if constexpr (POL) {
                if (a.Lpol) {  // O at point li: sum over the lane's four b, then over the rows
                    cd o = {0.0, 0.0};
#pragma unroll
                    for (int v = 0; v < 4 * H; ++v)
                        o = cfmac(ukn[v], cd{(double)d.u[v].x, (double)d.u[v].y}, o);
                    o.x += __shfl_xor(o.x, 16, 64);
                    o.y += __shfl_xor(o.y, 16, 64);
                    o.x += __shfl_xor(o.x, 32, 64);
                    o.y += __shfl_xor(o.y, 32, 64);
                    if (wave == 0 && lg == 0) sO[li] = o;
                }
            }
            __syncthreads();
            // Z[c, nu] = sum_sa E_q[sa, nu] Y[c, sa] and the rate terms
            if (pc >= 0) item_term(pc, ic, inu, d.em, d.fm, d.om, d.nbq, m);
            for (int it = tid + BT; it < 16 * nm; it += BT) {
                const int c = it / nm, nu = it - c * nm;
                if (g + c >= cnt) continue;
                const int q0 = sList[g + c];
                const int64_t q = (int64_t)q0 * NL + q12;
                const int64_t kq = kq_of(q0);
                item_term(q0, c, nu, a.eps[kq * nW + m], a.focc[kq * nW + m], a.omega[q * nm + nu],
                          a.nb[q * nm + nu], m);
            }
            __syncthreads();  // sY (and the list, after a band's last unit) are rewritten
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) gacc += __shfl_xor(gacc, o, 64);
    if (lane == 0) sRed[wave] = gacc;
    __syncthreads();
    if (tid == 0) {
        double tot;
        if constexpr (NWV == 4)
            tot = (sRed[0] + sRed[1]) + (sRed[2] + sRed[3]);
        else
            tot = sRed[0] + sRed[1];
        a.partial[(int64_t)st * a.n_qtiles + line] = tot;
    }
    if constexpr (LW) {
        if (a.lw) {  // (the last __syncthreads above ordered every sLW update)
            // only the live points' partials: the reduction reads those alone
            double* o = a.lw + ((int64_t)st * NL + line) * N0 * nm;
            for (int i = tid; i < N0 * nm; i += BT)
                if (sPm[i / nm]) o[i] = sLW[i];
        }
    }
}

size_t line_rates_lds(int W, int N0, int nm, bool f32, bool lw) {
    const int Wp = (W + 3) & ~3;
    return ((size_t)(N0 + 1) * (Wp + 1) + 16 * (size_t)nm) * (f32 ? sizeof(cf) : sizeof(cd)) +
           2 * (size_t)N0 * sizeof(uint32_t) +
           (lw ? sizeof(uint32_t) * (size_t)(N0 & 1) + (size_t)N0 * nm * sizeof(double) : 0);
}

// Columns of the factorised form, 4 waves x TN tiles of 16 (or 2 x 2 TN): one tile per mode index
// (nW <= 16), or two (16 < nW <= 32: a wave takes TN / 2 whole modes).
int line_rates_ncpad(int nm, int nW) {
    if (nW > 32 || nm > 32 || nm < 1 || nW < 1) return -1;
    if (nW <= 16) {
        const int tn = (nm + 3) / 4;
        return 64 * (tn == 5 ? 6 : (tn == 7 ? 8 : tn));
    }
    const int tn = 2 * ((nm + 3) / 4);  // even: whole modes per wave
    return 64 * (tn <= 8 ? tn : (tn <= 12 ? 12 : 16));
}

template <int TN, int KS, class C, int FEAT, int H = 1, int NWV = 4>
static hipError_t go_line(const RateArgs& a, int nst, hipStream_t s) {
    const size_t shm = line_rates_lds(a.W, a.mesh.n0, a.nm, sizeof(C) == sizeof(cf), a.lw != nullptr);
    if (shm > 64 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void*)line_rates_kernel<TN, KS, C, FEAT, H, NWV>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    const int64_t NL = (int64_t)a.mesh.n1 * a.mesh.n2;
    const int64_t groups = (NL + 7) / 8;
    const int chunk = (int)std::min<int64_t>(65535, 2147483647LL / (groups * 8));
    for (int s0 = 0; s0 < nst; s0 += chunk) {
        const int ns = nst - s0 < chunk ? nst - s0 : chunk;
        RateArgs b = a;
        b.T2 = reinterpret_cast<const C*>(a.T2) + (int64_t)s0 * a.W * NL * a.nc_pad;
        b.st_kmesh += s0;
        b.st_band += s0;
        b.st_row += s0;
        b.st_mlo += s0;
        b.st_mhi += s0;
        b.partial = a.partial + (int64_t)s0 * a.n_qtiles;
        if (a.terms) b.terms = a.terms + (int64_t)s0 * a.nq_mesh * a.nm;
        b.live = a.live + (int64_t)s0 * a.mesh.n0 * NL;
        b.line_bands = a.line_bands + (int64_t)s0 * NL;
        if (a.lw) b.lw = a.lw + (int64_t)s0 * NL * a.mesh.n0 * a.nm;
        b.n_states = ns;
        hipLaunchKernelGGL((line_rates_kernel<TN, KS, C, FEAT, H, NWV>),
                           dim3((unsigned)(groups * 8 * ns)), dim3(64 * NWV), shm, s, b);
    }
    return hipGetLastError();
}

template <class C>
static hipError_t line_rates(const RateArgs& a, int nst, hipStream_t s) {
    if (nst <= 0) return hipSuccess;
    if (a.n_qtiles != a.mesh.n1 * a.mesh.n2 || a.n_qtiles > 65535 || a.W > kMaxW ||
        line_rates_ncpad(a.nm, a.nW) != a.nc_pad || !a.live || !a.line_bands)
        return hipErrorInvalidValue;
    const bool pre = a.W <= 8;  // T2 rows fit two K steps: registers
    const int feat = (a.lw ? kLineLW : 0) | (a.Lpol ? kLinePol : 0) | (a.vel ? kLineVel : 0);
    if (feat && sizeof(C) != sizeof(cd)) return hipErrorInvalidValue;  // the extensions are FP64 only
    auto with_feat = [&](auto tn, auto ks) -> hipError_t {
        constexpr int TN = decltype(tn)::value, KS = decltype(ks)::value;
        if constexpr (sizeof(C) == sizeof(cd)) {
            switch (feat) {
                case 0: return go_line<TN, KS, C, 0>(a, nst, s);
                case kLineLW: return go_line<TN, KS, C, kLineLW>(a, nst, s);
                case kLinePol: return go_line<TN, KS, C, kLinePol>(a, nst, s);
                case kLineVel: return go_line<TN, KS, C, kLineVel>(a, nst, s);
                default: return go_line<TN, KS, C, kLineLW | kLinePol | kLineVel>(a, nst, s);
            }
        } else {
            return go_line<TN, KS, C, 0>(a, nst, s);
        }
    };
    using std::integral_constant;
    if (a.nW > 16) {  // two tiles per mode
        auto with_feat2 = [&](auto tn, auto ks) -> hipError_t {
            constexpr int TN = decltype(tn)::value, KS = decltype(ks)::value;
            if constexpr (sizeof(C) == sizeof(cd)) {
                switch (feat) {
                    case 0: return go_line<TN, KS, C, 0, 2>(a, nst, s);
                    case kLineLW: return go_line<TN, KS, C, kLineLW, 2>(a, nst, s);
                    case kLinePol: return go_line<TN, KS, C, kLinePol, 2>(a, nst, s);
                    case kLineVel: return go_line<TN, KS, C, kLineVel, 2>(a, nst, s);
                    default: return go_line<TN, KS, C, kLineLW | kLinePol | kLineVel, 2>(a, nst, s);
                }
            } else {
                return go_line<TN, KS, C, 0, 2>(a, nst, s);
            }
        };
        switch (a.nc_pad / 64) {
            case 2:
                if (pre && feat == 0) return go_line<4, 2, C, 0, 2, 2>(a, nst, s);
                return pre ? with_feat2(integral_constant<int, 2>{}, integral_constant<int, 2>{})
                           : with_feat2(integral_constant<int, 2>{}, integral_constant<int, 0>{});
            case 4:
                // (FP32 only: the FP64 form would spill)
                if (pre && feat == 0 && sizeof(C) == sizeof(cf)) return go_line<8, 2, C, 0, 2, 2>(a, nst, s);
                return pre ? with_feat2(integral_constant<int, 4>{}, integral_constant<int, 2>{})
                           : with_feat2(integral_constant<int, 4>{}, integral_constant<int, 0>{});
            case 6:
                if (feat == 0) return go_line<12, 0, C, 0, 2, 2>(a, nst, s);
                return with_feat2(integral_constant<int, 6>{}, integral_constant<int, 0>{});
            case 8:
                if (feat == 0) return go_line<16, 0, C, 0, 2, 2>(a, nst, s);
                return with_feat2(integral_constant<int, 8>{}, integral_constant<int, 0>{});
            case 12: return with_feat2(integral_constant<int, 12>{}, integral_constant<int, 0>{});
            case 16: return with_feat2(integral_constant<int, 16>{}, integral_constant<int, 0>{});
            default: return hipErrorInvalidValue;
        }
    }
    switch (a.nc_pad / 64) {
        case 1: return pre ? with_feat(integral_constant<int, 1>{}, integral_constant<int, 2>{})
                           : with_feat(integral_constant<int, 1>{}, integral_constant<int, 0>{});
        case 2:
            if (pre && feat == 0) return go_line<4, 2, C, 0, 1, 2>(a, nst, s);
            return pre ? with_feat(integral_constant<int, 2>{}, integral_constant<int, 2>{})
                       : with_feat(integral_constant<int, 2>{}, integral_constant<int, 0>{});
        case 3:
            if (pre && feat == 0) return go_line<6, 2, C, 0, 1, 2>(a, nst, s);
            return pre ? with_feat(integral_constant<int, 3>{}, integral_constant<int, 2>{})
                       : with_feat(integral_constant<int, 3>{}, integral_constant<int, 0>{});
        case 4:
            // the plain rates: two waves of eight tiles, six work-groups per CU
            if (pre && feat == 0) return go_line<8, 2, C, 0, 1, 2>(a, nst, s);
            if constexpr (sizeof(C) == sizeof(cd)) {
                if (pre && feat == kLineLW) return go_line<8, 2, C, kLineLW, 1, 2>(a, nst, s);
                if (pre && feat == kLinePol) return go_line<8, 2, C, kLinePol, 1, 2>(a, nst, s);
                if (pre && feat == kLineVel) return go_line<8, 2, C, kLineVel, 1, 2>(a, nst, s);
            }
            return pre ? with_feat(integral_constant<int, 4>{}, integral_constant<int, 2>{})
                       : with_feat(integral_constant<int, 4>{}, integral_constant<int, 0>{});
        case 6:
            if (feat == 0) return go_line<12, 0, C, 0, 1, 2>(a, nst, s);
            return with_feat(integral_constant<int, 6>{}, integral_constant<int, 0>{});
        case 8:
            if (feat == 0) return go_line<16, 0, C, 0, 1, 2>(a, nst, s);
            return with_feat(integral_constant<int, 8>{}, integral_constant<int, 0>{});
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_line_rates(const RateArgs& a, int nst, hipStream_t s) {
    return line_rates<cd>(a, nst, s);
}
hipError_t launch_line_rates_f32(const RateArgs& a, int nst, hipStream_t s) {
    return line_rates<cf>(a, nst, s);
}

}  // namespace phx
