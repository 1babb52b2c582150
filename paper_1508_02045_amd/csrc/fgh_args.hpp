// fgh_args.hpp -- kernel-argument structures of the passes and the per-point coefficient
// helpers shared by the generic and the size-specialised pass kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "fgh_fft.hpp"
#include "fgh_internal.hpp"

namespace fgh {

// ------------------------------------------------------------------------------------------
// Coefficient helpers: z = A(pt) u with A as the passes see it (eq:A, eq:GaNi, eq:Ga_eval).
// ------------------------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void sym_mul(const T* a, const T* u, T* z)
{
    if (D == 2) {  // a00 a01 a11
        z[0] = a[0] * u[0] + a[1] * u[1];
        z[1] = a[1] * u[0] + a[2] * u[1];
    } else {       // a00 a01 a02 a11 a12 a22
        z[0] = a[0] * u[0] + a[1] * u[1] + a[2] * u[2];
        z[1] = a[1] * u[0] + a[3] * u[1] + a[4] * u[2];
        z[2] = a[2] * u[0] + a[4] * u[1] + a[5] * u[2];
    }
}

template <int D>
constexpr int ncoef_of() { return D == 2 ? 3 : 6; }

// Load the packed coefficients of point pt into a[] (AK_ISO gives a scalar in a[0]).
template <typename T, int D, int AK>
__device__ __forceinline__ void load_coef(const CoefArgs& A, const T* tab, long long pt, long long npts, T* a)
{
    if (AK == AK_ISO) {
        a[0] = static_cast<const T*>(A.coef)[pt];
    } else if (AK == AK_PHASE) {
        const int ph = A.phase[pt];
#pragma unroll
        for (int q = 0; q < ncoef_of<D>(); q++) a[q] = tab[ph * 6 + q];
    } else {
        const T* c = static_cast<const T*>(A.coef);
#pragma unroll
        for (int q = 0; q < ncoef_of<D>(); q++) a[q] = c[q * npts + pt];
    }
}

template <typename T, int D, int AK>
__device__ __forceinline__ void mul_A(const T* a, const T* u, T* z)
{
    if (AK == AK_ISO) {
#pragma unroll
        for (int c = 0; c < D; c++) z[c] = a[0] * u[c];
    } else {
        sym_mul<T, D>(a, u, z);
    }
}

// Solve (A + w I) v = rhs at one point for packed symmetric A (closed-form inverse).
template <typename T, int D>
__device__ __forceinline__ void sym_shift_solve(const T* a, T w, const T* rhs, T* v)
{
    if (D == 2) {
        const T m00 = a[0] + w, m01 = a[1], m11 = a[2] + w;
        const T det = m00 * m11 - m01 * m01;
        v[0] = (m11 * rhs[0] - m01 * rhs[1]) / det;
        v[1] = (-m01 * rhs[0] + m00 * rhs[1]) / det;
    } else {
        const T m00 = a[0] + w, m01 = a[1], m02 = a[2], m11 = a[3] + w, m12 = a[4], m22 = a[5] + w;
        const T c00 = m11 * m22 - m12 * m12;
        const T c01 = m02 * m12 - m01 * m22;
        const T c02 = m01 * m12 - m02 * m11;
        const T c11 = m00 * m22 - m02 * m02;
        const T c12 = m01 * m02 - m00 * m12;
        const T c22 = m00 * m11 - m01 * m01;
        const T det = m00 * c00 + m01 * c01 + m02 * c02;
        v[0] = (c00 * rhs[0] + c01 * rhs[1] + c02 * rhs[2]) / det;
        v[1] = (c01 * rhs[0] + c11 * rhs[1] + c12 * rhs[2]) / det;
        v[2] = (c02 * rhs[0] + c12 * rhs[1] + c22 * rhs[2]) / det;
    }
}

template <typename T>
struct FirstArgs {
    const int* done;  // the loop's stop flag (nullptr: always run)
    Geo g;
    Axis ax;
    int rpb, npen;
    const T* x;
    T* p;
    const T* r;
    // OP_AP_CG with a deferred iterate update: x += alpha p with the loop's current alpha and the
    // p on entry, before p is replaced (nullptr: x is updated elsewhere)
    T* xd;
    const Scalars* sc;
    double E[3];
    double omega;
    CoefArgs A;
    cpx<T>* out;
    const cpx<T>* twg;
};

template <typename T>
struct AxisArgs {
    const int* done;  // the loop's stop flag (nullptr: always run)
    Axis ax;
    int nin, nout;          // stored counts along the axis
    int bin, bout;          // 1: stored index is a band index (frequency signed(s, n)), 0: position
    int inner, P, ntiles;
    long long in_os, out_os, in_cs, out_cs;
    const cpx<T>* in;
    cpx<T>* out;
    const cpx<T>* twg;
    Scalars* red_sc;          // non-null: workgroup 0 completes a deferred loop reduction first
    const double* partials;
};

template <typename T>
struct MidArgs {
    const int* done;  // the loop's stop flag (nullptr: always run)
    Axis ax;
    int B0, cols, Hb, B1, P, ntiles;
    int ys;        // specialised kernel: LDS stride of a column (complex elements, >= L)
    long long cs;
    double scale;  // 1 / |grid| (the forward DFT factor of eq:DFT)
    cpx<T>* buf;
    const cpx<T>* twg;
};

template <typename T>
struct LastArgs {
    const int* done;  // the loop's stop flag (nullptr: always run)
    const Scalars* sc;  // Chebyshev alpha, beta (device) when non-null
    Geo g;
    Axis ax;
    int rpb, npen;
    const cpx<T>* in;
    T* y;
    T* x;
    T* r;
    T* p;
    T* q;
    const T* src;
    double E[3];
    double omega, alpha, beta, sgn;
    CoefArgs A;
    double* partials;
    const cpx<T>* twg;
    cpx<T>* out;    // fused last + first pass: the next body's first spectrum (rows of this tile)
    Scalars* defer_sc;  // non-null: the loop reduction redop of these partials is left to the next body
    int redop;
};

}  // namespace fgh
