// Shared device/host definitions of the gfx950 el-ph library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/phoebe_gpu.h"

namespace phx {

// ---------------------------------------------------------------------------
// Units (CODATA 2018).  Energies eV, lengths A, masses amu.
//   hbar omega = C_OMEGA sqrt(lambda), lambda in eV/(A^2 amu)
//   l^2 = C_PH / (2 M hbar omega) in A^2
// ---------------------------------------------------------------------------
constexpr double kHbar = 1.054571817e-34;      // J s
constexpr double kEv = 1.602176634e-19;        // J
constexpr double kAmu = 1.66053906660e-27;     // kg
constexpr double kAng = 1.0e-10;               // m
// C_OMEGA = hbar sqrt(eV / (A^2 amu)) / eV ; C_PH = hbar^2 / (amu A^2) / eV
constexpr double kCPh = kHbar * kHbar / (kAmu * kAng * kAng) / kEv;
// sqrt is not constexpr: C_OMEGA^2 = C_PH (same combination), so C_OMEGA = sqrt(C_PH)
inline double c_omega() { return __builtin_sqrt(kCPh); }

constexpr double kPi = 3.14159265358979323846;

struct cd {
    double x, y;
};

__host__ __device__ inline cd cmul(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline cd cmulc(cd a, cd b) {  // conj(a) * b
    return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__host__ __device__ inline cd cadd(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cd cfma(cd a, cd b, cd c) {  // a*b + c
    return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
__host__ __device__ inline cd cfmac(cd a, cd b, cd c) {  // conj(a)*b + c
    return {fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y))};
}
__host__ __device__ inline double cabs2(cd a) { return a.x * a.x + a.y * a.y; }

struct cf {
    float x, y;
};
__host__ __device__ inline cf cfma(cf a, cf b, cf c) {  // a*b + c, FP32
    return {fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y))};
}
__host__ __device__ inline double cabs2(cf a) { return (double)a.x * a.x + (double)a.y * a.y; }

// complex value in the working type C (cd or cf) from an FP64 one
template <class C>
__host__ __device__ inline C to_c(cd v) {
    return C{(decltype(C::x))v.x, (decltype(C::x))v.y};
}

// e^{i 2 pi t} for t already reduced to [-1, 1)
__device__ inline cd expi2pi(double t) {
    double s, c;
    sincospi(2.0 * t, &s, &c);
    return {c, s};
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

// One complex element of an LDS (or global) array whose elements sit at their
// natural vector alignment (16 bytes for cd, 8 for cf): one 128-bit (64-bit)
// access per lane instead of two halves.  The structs themselves only promise
// the alignment of their scalar members.
__device__ inline cd ld_vec(const cd* p) {
    const d2 v = *reinterpret_cast<const d2*>(p);
    return cd{v.x, v.y};
}
__device__ inline cf ld_vec(const cf* p) {
    const f2 v = *reinterpret_cast<const f2*>(p);
    return cf{v.x, v.y};
}
__device__ inline void st_vec(cd* p, cd v) { *reinterpret_cast<d2*>(p) = d2{v.x, v.y}; }

// C += A B for complex 16 x 16 x 4 tiles on v_mfma_f64_16x16x4f64: four real
// products; (ar, ai) this lane's A entry, (br, bi) its B entry
__device__ inline void cmfma_f64(d4& cr, d4& ci, double ar, double ai, double br, double bi) {
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, cr, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, ci, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, ci, 0, 0, 0);
}
__device__ inline void st_vec(cf* p, cf v) { *reinterpret_cast<f2*>(p) = f2{v.x, v.y}; }

// Mesh helpers: linear index (i0 N1 + i1) N2 + i2
struct Mesh {
    int n0, n1, n2;
};
__host__ __device__ inline void mesh_triple(int64_t idx, Mesh m, int& i0, int& i1, int& i2) {
    i2 = (int)(idx % m.n2);
    idx /= m.n2;
    i1 = (int)(idx % m.n1);
    i0 = (int)(idx / m.n1);
}
__host__ __device__ inline int64_t mesh_linear(int i0, int i1, int i2, Mesh m) {
    return ((int64_t)i0 * m.n1 + i1) * m.n2 + i2;
}

}  // namespace phx
