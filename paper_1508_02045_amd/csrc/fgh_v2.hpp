// fgh_v2.hpp -- size-specialised passes: compile-time length L = L1 * L2, register-resident DFTs.
//
// Index split (n = n1 + L1 n2, k = k2 + L2 k1):
//   X[k2 + L2 k1] = sum_{n1} W_L1^{n1 k1} W_L^{n1 k2} sum_{n2} W_L2^{n2 k2} x[n1 + L1 n2]
// Step A: per n1, an L2-point DFT of the stride-L1 subsequence, times W_L^{n1 k2}; step B: per
// k2, an L1-point DFT.  Both DFTs run in registers (compound sizes recurse on the same split with
// compile-time roots), so a pass moves its tile global -> registers -> LDS -> registers -> global:
// one LDS exchange and one barrier per pass (two in the middle pass, whose forward step B, the
// Fourier multiplier and the inverse step B all stay in registers).
#pragma once
#include <hip/hip_runtime.h>

#include "fgh_args.hpp"

namespace fgh {

constexpr int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; p++)
        if (n % p == 0) return p;
    return n;
}

// exp(-+2 pi i m / R) with m, R compile-time after unrolling (the compiler folds the trig).
template <typename T, int R, bool INV>
__device__ __forceinline__ cpx<T> croot(int m)
{
    const double a = 6.283185307179586476925286766559 * double(m % R) / double(R);
    return {T(cos(a)), T(INV ? sin(a) : -sin(a))};
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void reg_dft(cpx<T>* v);

// Direct DFT for a prime R > 7.
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_direct(cpx<T>* v)
{
    cpx<T> out[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
        cpx<T> acc = v[0];
#pragma unroll
        for (int n = 1; n < R; n++) acc = acc + cmul(v[n], croot<T, R, INV>(n * k));
        out[k] = acc;
    }
#pragma unroll
    for (int k = 0; k < R; k++) v[k] = out[k];
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void reg_dft(cpx<T>* v)
{
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 3 || R == 5 || R == 7) {
        dft_small<T, R, INV>(v);
    } else if constexpr (smallest_factor(R) == R) {
        dft_direct<T, R, INV>(v);
    } else {
        constexpr int R1 = smallest_factor(R);
        constexpr int R2 = R / R1;
        cpx<T> y[R];
#pragma unroll
        for (int n1 = 0; n1 < R1; n1++) {
            cpx<T> s[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; n2++) s[n2] = v[n1 + R1 * n2];
            reg_dft<T, R2, INV>(s);
#pragma unroll
            for (int k2 = 0; k2 < R2; k2++) y[n1 * R2 + k2] = (n1 * k2 == 0) ? s[k2] : cmul(s[k2], croot<T, R, INV>(n1 * k2));
        }
#pragma unroll
        for (int k2 = 0; k2 < R2; k2++) {
            cpx<T> s[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; n1++) s[n1] = y[n1 * R2 + k2];
            reg_dft<T, R1, INV>(s);
#pragma unroll
            for (int k1 = 0; k1 < R1; k1++) v[k2 + R2 * k1] = s[k1];
        }
    }
}

// ------------------------------------------------------------------------------------------
// Runtime-kind coefficient helpers (the kind is uniform across the launch).
// ------------------------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void coef_mul_rt(const CoefArgs& A, const T* tab, long long pt, long long npts,
                                            const T* u, T* z)
{
    if (A.kind == AK_ISO) {
        const T a = static_cast<const T*>(A.coef)[pt];
#pragma unroll
        for (int c = 0; c < D; c++) z[c] = a * u[c];
    } else if (A.kind == AK_PHASE) {
        sym_mul<T, D>(tab + 6 * A.phase[pt], u, z);
    } else {
        T co[6];
        const T* cc = static_cast<const T*>(A.coef);
#pragma unroll
        for (int q = 0; q < ncoef_of<D>(); q++) co[q] = cc[q * npts + pt];
        sym_mul<T, D>(co, u, z);
    }
}

// (A + w I)^{-1} v at one point.
template <typename T, int D>
__device__ __forceinline__ void coef_shift_solve_rt(const CoefArgs& A, const T* tabinv, T w, long long pt,
                                                    long long npts, const T* v, T* xn)
{
    if (A.kind == AK_ISO) {
        const T av = static_cast<const T*>(A.coef)[pt];
#pragma unroll
        for (int c = 0; c < D; c++) xn[c] = v[c] / (av + w);
    } else if (A.kind == AK_PHASE) {
        sym_mul<T, D>(tabinv + 6 * A.phase[pt], v, xn);
    } else {
        T co[6];
        const T* cc = static_cast<const T*>(A.coef);
#pragma unroll
        for (int q = 0; q < ncoef_of<D>(); q++) co[q] = cc[q * npts + pt];
        sym_shift_solve<T, D>(co, w, v, xn);
    }
}

// First-pass operand z at one point (FirstOp, runtime).
template <typename T, int D>
__device__ __forceinline__ void first_operand(const FirstArgs<T>& a, int op, const T* tab, T beta, long long pt,
                                              T* z)
{
    const long long npts = a.g.npts;
    T u[D];
#pragma unroll
    for (int c = 0; c < D; c++) {
        if (op == OP_AX)
            u[c] = a.x[c * npts + pt] + T(a.E[c]);
        else if (op == OP_E)
            u[c] = T(a.E[c]);
        else if (op == OP_AP_CG) {
            const T pn = a.r[c * npts + pt] + beta * a.p[c * npts + pt];
            a.p[c * npts + pt] = pn;
            u[c] = pn;
        } else
            u[c] = a.x[c * npts + pt];
    }
    if (op == OP_ID) {
#pragma unroll
        for (int c = 0; c < D; c++) z[c] = u[c];
        return;
    }
    coef_mul_rt<T, D>(a.A, tab, pt, npts, u, z);
    if (op == OP_EM) {
#pragma unroll
        for (int c = 0; c < D; c++) z[c] -= T(a.omega) * u[c];
    }
}

// Solver epilogue at one point (Epi, runtime); returns the point's contribution to the sum.
template <typename T, int D>
__device__ __forceinline__ double last_epilogue(const LastArgs<T>& a, int epi, const T* tabinv, long long pt,
                                                const T* y)
{
    const long long npts = a.g.npts;
    double acc = 0.0;
    if (epi == EPI_STORE) {
#pragma unroll
        for (int c = 0; c < D; c++) {
            const T v = T(a.sgn) * y[c];
            a.y[c * npts + pt] = v;
            acc += double(v) * double(v);
        }
    } else if (epi == EPI_RICH) {
#pragma unroll
        for (int c = 0; c < D; c++) {
            const T s = T(-a.omega) * y[c];
            a.x[c * npts + pt] += s;
            acc += double(s) * double(s);
        }
    } else if (epi == EPI_CG) {
#pragma unroll
        for (int c = 0; c < D; c++) {
            a.q[c * npts + pt] = y[c];
            acc += double(y[c]) * double(a.p[c * npts + pt]);
        }
    } else if (epi == EPI_CHEB) {
        const T al = T(a.alpha), be = T(a.beta);
#pragma unroll
        for (int c = 0; c < D; c++) {
            const long long o = c * npts + pt;
            const T pv = a.p[o];
            const T rv = a.r[o] - al * y[c];
            a.r[o] = rv;
            a.x[o] += al * pv;
            a.p[o] = rv - be * pv;
            acc += double(rv) * double(rv);
        }
    } else {  // EPI_EM
        const T w = T(a.omega);
        T v[D], xn[D];
#pragma unroll
        for (int c = 0; c < D; c++) v[c] = a.src ? y[c] : y[c] + T(2.0 * a.omega * a.E[c]);
        coef_shift_solve_rt<T, D>(a.A, tabinv, w, pt, npts, v, xn);
#pragma unroll
        for (int c = 0; c < D; c++) {
            const long long o = c * npts + pt;
            if (a.src) xn[c] += a.src[o];
            const T s = xn[c] - a.x[o];
            a.x[o] = xn[c];
            acc += double(s) * double(s);
        }
    }
    return acc;
}

// Frequency position pos of an FFT of length L in the band of B frequencies?  Band index out.
__device__ __forceinline__ bool band_index(int pos, int L, int B, int* s)
{
    const int k = signed_index(pos, L);
    const int ak = k < 0 ? -k : k;
    if (2 * ak >= B) return false;
    *s = k < 0 ? k + B : k;
    return true;
}

// ------------------------------------------------------------------------------------------
// Pass 1 (rows of the last axis): z = A(x) op x, forward DFT, keep k < Hb.
// Step A jobs (row r, n1) hold the d components; step B jobs (r, c, k2).
// ------------------------------------------------------------------------------------------
template <typename T, int D, int L1, int L2>
__global__ __launch_bounds__(kThreads) void k2_first(FirstArgs<T> a, int op)
{
    constexpr int L = L1 * L2;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* Y = tw + L;
    T* tab = reinterpret_cast<T*>(Y + a.rpb * D * L);
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    if (a.A.kind == AK_PHASE)
        for (int m = threadIdx.x; m < kMaxPhases * 6; m += blockDim.x) tab[m] = T(a.A.tab[m / 6][m % 6]);
    __syncthreads();
    const long long row0 = (long long)blockIdx.x * a.rpb;
    const T beta = (op == OP_AP_CG) ? T(a.sc->beta) : T(0);
    for (int job = threadIdx.x; job < a.rpb * L1; job += blockDim.x) {
        const int r = job / L1;
        const int n1 = job - r * L1;
        const long long row = row0 + r;
        cpx<T> s[D][L2];
        if (row < a.g.rows) {
#pragma unroll
            for (int n2 = 0; n2 < L2; n2++) {
                T z[D];
                first_operand<T, D>(a, op, tab, beta, row * L + n1 + L1 * n2, z);
#pragma unroll
                for (int c = 0; c < D; c++) s[c][n2] = {z[c], T(0)};
            }
        } else {
#pragma unroll
            for (int c = 0; c < D; c++)
#pragma unroll
                for (int n2 = 0; n2 < L2; n2++) s[c][n2] = {T(0), T(0)};
        }
#pragma unroll
        for (int c = 0; c < D; c++) {
            reg_dft<T, L2, false>(s[c]);
            cpx<T>* y = Y + (r * D + c) * L + n1 * L2;
            int m = 0;
#pragma unroll
            for (int k2 = 0; k2 < L2; k2++) {
                y[k2] = k2 ? cmul(s[c][k2], tw[m]) : s[c][k2];
                m += n1;
                if (m >= L) m -= L;
            }
        }
    }
    __syncthreads();
    const int Hb = a.g.Hb;
    for (int job = threadIdx.x; job < a.rpb * D * L2; job += blockDim.x) {
        const int rc = job / L2;
        const int k2 = job - rc * L2;
        const int r = rc / D;
        const int c = rc - r * D;
        const long long row = row0 + r;
        cpx<T> s[L1];
        const cpx<T>* y = Y + rc * L + k2;
#pragma unroll
        for (int n1 = 0; n1 < L1; n1++) s[n1] = y[n1 * L2];
        reg_dft<T, L1, false>(s);
        if (row < a.g.rows) {
            cpx<T>* out = a.out + c * a.g.s1 + row * Hb;
#pragma unroll
            for (int k1 = 0; k1 < L1; k1++) {
                const int k = k2 + L2 * k1;
                if (k < Hb) out[k] = s[k1];
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Strided axis pass (3D axis 1), one component per workgroup, tile of P columns.
// ------------------------------------------------------------------------------------------
template <typename T, int L1, int L2, bool INV>
__global__ __launch_bounds__(kThreads) void k2_axis(AxisArgs<T> a, int B)
{
    constexpr int L = L1 * L2;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* Y = tw + L;
    const int P = a.P;
    const int tile = blockIdx.x, o = blockIdx.y, c = blockIdx.z;
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    __syncthreads();
    const cpx<T>* in = a.in + c * a.in_cs + o * a.in_os;
    cpx<T>* out = a.out + c * a.out_cs + o * a.out_os;
    for (int job = threadIdx.x; job < P * L1; job += blockDim.x) {
        const int n1 = job / P;
        const int p = job - n1 * P;
        const int j = tile * P + p;
        cpx<T> s[L2];
#pragma unroll
        for (int n2 = 0; n2 < L2; n2++) {
            const int pos = n1 + L1 * n2;
            int si = pos;
            bool ok = j < a.inner;
            if (a.bin) ok = ok && band_index(pos, L, B, &si);
            s[n2] = ok ? in[(long long)si * a.inner + j] : cpx<T>{T(0), T(0)};
        }
        reg_dft<T, L2, INV>(s);
        cpx<T>* y = Y + p * L + n1 * L2;
        int m = 0;
#pragma unroll
        for (int k2 = 0; k2 < L2; k2++) {
            y[k2] = k2 ? cmul(s[k2], INV ? conj(tw[m]) : tw[m]) : s[k2];
            m += n1;
            if (m >= L) m -= L;
        }
    }
    __syncthreads();
    for (int job = threadIdx.x; job < P * L2; job += blockDim.x) {
        const int k2 = job / P;
        const int p = job - k2 * P;
        const int j = tile * P + p;
        cpx<T> s[L1];
        const cpx<T>* y = Y + p * L + k2;
#pragma unroll
        for (int n1 = 0; n1 < L1; n1++) s[n1] = y[n1 * L2];
        reg_dft<T, L1, INV>(s);
        if (j < a.inner) {
#pragma unroll
            for (int k1 = 0; k1 < L1; k1++) {
                const int pos = k2 + L2 * k1;
                int so = pos;
                if (a.bout && !band_index(pos, L, B, &so)) continue;
                out[(long long)so * a.inner + j] = s[k1];
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Middle pass along axis 0 (all components, in place): forward step A -> LDS -> forward step B,
// multiplier and inverse step B in registers -> LDS -> inverse step A.
// ------------------------------------------------------------------------------------------
template <typename T, int D, int L1, int L2>
__global__ __launch_bounds__(kThreads) void k2_middle(MidArgs<T> a, int mult)
{
    constexpr int L = L1 * L2;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* Y = tw + L;
    const int P = a.P;
    const int PL = P * L;
    const int tile = blockIdx.x;
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    __syncthreads();
    // forward step A: jobs (c, n1, p), p fastest
    for (int job = threadIdx.x; job < D * P * L1; job += blockDim.x) {
        const int cn = job / P;
        const int p = job - cn * P;
        const int c = cn / L1;
        const int n1 = cn - c * L1;
        const int j = tile * P + p;
        const cpx<T>* in = a.buf + c * a.cs + j;
        cpx<T> s[L2];
#pragma unroll
        for (int n2 = 0; n2 < L2; n2++)
            s[n2] = (j < a.cols) ? in[(long long)(n1 + L1 * n2) * a.cols] : cpx<T>{T(0), T(0)};
        reg_dft<T, L2, false>(s);
        cpx<T>* y = Y + c * PL + p * L + n1 * L2;
        int m = 0;
#pragma unroll
        for (int k2 = 0; k2 < L2; k2++) {
            y[k2] = k2 ? cmul(s[k2], tw[m]) : s[k2];
            m += n1;
            if (m >= L) m -= L;
        }
    }
    __syncthreads();
    // forward step B, multiplier, inverse step B: jobs (k2, p)
    const T scale = T(a.scale);
    for (int job = threadIdx.x; job < P * L2; job += blockDim.x) {
        const int k2 = job / P;
        const int p = job - k2 * P;
        const int j = tile * P + p;
        cpx<T> s[D][L1];
#pragma unroll
        for (int c = 0; c < D; c++) {
            const cpx<T>* y = Y + c * PL + p * L + k2;
#pragma unroll
            for (int n1 = 0; n1 < L1; n1++) s[c][n1] = y[n1 * L2];
            reg_dft<T, L1, false>(s[c]);
        }
        int kv1 = 0, kv2 = 0;
        if (D == 2) {
            kv1 = j;
        } else {
            const int kb1 = j / a.Hb;
            kv1 = signed_index(kb1, a.B1);
            kv2 = j - kb1 * a.Hb;
        }
        const bool colok = j < a.cols;
#pragma unroll
        for (int k1 = 0; k1 < L1; k1++) {
            const int pos = k2 + L2 * k1;
            const int k0 = signed_index(pos, L);
            const bool inband = colok && (2 * (k0 < 0 ? -k0 : k0) < a.B0);
            const double kk = double(k0) * k0 + double(kv1) * kv1 + double(kv2) * kv2;
            cpx<T> z[D];
#pragma unroll
            for (int c = 0; c < D; c++) z[c] = s[c][k1];
            if (!inband) {
#pragma unroll
                for (int c = 0; c < D; c++) s[c][k1] = {T(0), T(0)};
            } else if (kk == 0.0) {
#pragma unroll
                for (int c = 0; c < D; c++) s[c][k1] = (mult == MULT_EM) ? scale * z[c] : cpx<T>{T(0), T(0)};
            } else {
                const T kvec[3] = {T(k0), T(kv1), T(kv2)};
                cpx<T> kz = {T(0), T(0)};
#pragma unroll
                for (int c = 0; c < D; c++) kz = kz + kvec[c] * z[c];
                const T inv = T(1.0 / kk);
#pragma unroll
                for (int c = 0; c < D; c++) {
                    const cpx<T> gz = (kvec[c] * inv) * kz;
                    s[c][k1] = (mult == MULT_G) ? scale * gz : scale * (z[c] - T(2) * gz);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < D; c++) {
            reg_dft<T, L1, true>(s[c]);
            cpx<T>* y = Y + c * PL + p * L + k2;
            int m = 0;
#pragma unroll
            for (int n1 = 0; n1 < L1; n1++) {
                y[n1 * L2] = n1 ? cmul(s[c][n1], conj(tw[m])) : s[c][n1];
                m += k2;
                if (m >= L) m -= L;
            }
        }
    }
    __syncthreads();
    // inverse step A: jobs (c, n1, p)
    for (int job = threadIdx.x; job < D * P * L1; job += blockDim.x) {
        const int cn = job / P;
        const int p = job - cn * P;
        const int c = cn / L1;
        const int n1 = cn - c * L1;
        const int j = tile * P + p;
        cpx<T> s[L2];
        const cpx<T>* y = Y + c * PL + p * L + n1 * L2;
#pragma unroll
        for (int k2 = 0; k2 < L2; k2++) s[k2] = y[k2];
        reg_dft<T, L2, true>(s);
        if (j < a.cols) {
            cpx<T>* outp = a.buf + c * a.cs + j;
#pragma unroll
            for (int n2 = 0; n2 < L2; n2++) outp[(long long)(n1 + L1 * n2) * a.cols] = s[n2];
        }
    }
}

// ------------------------------------------------------------------------------------------
// Last pass: inverse step B from the half spectra (Hermitian completion), LDS, inverse step A
// with the d components of a point together, solver epilogue.
// ------------------------------------------------------------------------------------------
template <typename T, int D, int L1, int L2>
__global__ __launch_bounds__(kThreads) void k2_last(LastArgs<T> a, int epi)
{
    constexpr int L = L1 * L2;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* Y = tw + L;
    T* tab = reinterpret_cast<T*>(Y + a.rpb * D * L);
    __shared__ double red[kThreads / 64];
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    if (epi == EPI_EM && a.A.kind == AK_PHASE)
        for (int m = threadIdx.x; m < kMaxPhases * 6; m += blockDim.x) tab[m] = T(a.A.tab_inv[m / 6][m % 6]);
    __syncthreads();
    const long long row0 = (long long)blockIdx.x * a.rpb;
    const int Hb = a.g.Hb;
    for (int job = threadIdx.x; job < a.rpb * D * L2; job += blockDim.x) {
        const int rc = job / L2;
        const int k2 = job - rc * L2;
        const int r = rc / D;
        const int c = rc - r * D;
        const long long row = row0 + r;
        cpx<T> s[L1];
        const cpx<T>* in = a.in + c * a.g.s1 + row * Hb;
        const bool ok = row < a.g.rows;
#pragma unroll
        for (int k1 = 0; k1 < L1; k1++) {
            const int k = k2 + L2 * k1;
            cpx<T> v = {T(0), T(0)};
            if (ok) {
                if (k < Hb)
                    v = in[k];
                else if (L - k < Hb)
                    v = conj(in[L - k]);
            }
            s[k1] = v;
        }
        reg_dft<T, L1, true>(s);
        cpx<T>* y = Y + rc * L + k2;
        int m = 0;
#pragma unroll
        for (int n1 = 0; n1 < L1; n1++) {
            y[n1 * L2] = n1 ? cmul(s[n1], conj(tw[m])) : s[n1];
            m += k2;
            if (m >= L) m -= L;
        }
    }
    __syncthreads();
    double acc = 0.0;
    for (int job = threadIdx.x; job < a.rpb * L1; job += blockDim.x) {
        const int r = job / L1;
        const int n1 = job - r * L1;
        const long long row = row0 + r;
        cpx<T> s[D][L2];
#pragma unroll
        for (int c = 0; c < D; c++) {
            const cpx<T>* y = Y + (r * D + c) * L + n1 * L2;
#pragma unroll
            for (int k2 = 0; k2 < L2; k2++) s[c][k2] = y[k2];
            reg_dft<T, L2, true>(s[c]);
        }
        if (row < a.g.rows) {
#pragma unroll
            for (int n2 = 0; n2 < L2; n2++) {
                T yv[D];
#pragma unroll
                for (int c = 0; c < D; c++) yv[c] = s[c][n2].x;
                acc += last_epilogue<T, D>(a, epi, tab, row * L + n1 + L1 * n2, yv);
            }
        }
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = tot;
}

// Lengths with a specialised kernel, and their split for the row passes (first/last: step A
// holds d x L2 values) and the column passes (axis/middle: step B holds d x L1 values).
struct Split {
    int L, row_L1, row_L2, col_L1, col_L2;
};
constexpr Split kSplits[] = {
    {45, 9, 5, 5, 9},    {63, 7, 9, 7, 9},     {81, 9, 9, 9, 9},   {125, 25, 5, 5, 25},
    {135, 15, 9, 9, 15}, {243, 27, 9, 9, 27},
};

inline bool v2_supported(int L)
{
    for (const Split& s : kSplits)
        if (s.L == L) return true;
    return false;
}

}  // namespace fgh
