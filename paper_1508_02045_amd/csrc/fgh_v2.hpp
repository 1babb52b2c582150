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

// 1 / v for an exact positive integer v: the hardware reciprocal, refined by one Newton step in
// double precision (relative error a few units in the last place).
__device__ __forceinline__ float recip_int(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double recip_int(double v)
{
    const double r = __builtin_amdgcn_rcp(v);
    return fma(fma(-v, r, 1.0), r, r);
}

// Workgroup barrier that orders LDS accesses only.  Threads of one launch exchange data through
// LDS alone, so global loads issued before the barrier (prefetches of the next tile) stay in
// flight across it, and global stores are not waited for.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void end_body(Scalars* s, double v)
{
    s->m += 1;
    const double q = sqrt(v / s->npts);
    s->last = q;
    if (!(v == v) || v > 1.0e300 || (s->blowup > 0.0 && q > s->blowup))
        s->done = 3;
    else if (s->thr >= 0.0 && q <= s->thr)
        s->done = 1;
    else if (s->m >= s->limit)
        s->done = 2;
}

// The scalar update that ends a loop reduction (RedOp) from its total.
__device__ __forceinline__ void apply_redop(Scalars* s, int op, double tot)
{
    s->total = tot;
    if (op == RED_CG_ALPHA) {
        s->qp = tot;
        s->alpha = s->rr / tot;
    } else if (op == RED_CG_END) {
        s->rr_new = tot;
        s->beta = tot / s->rr;
        s->rr = tot;
        end_body(s, tot);
    } else if (op == RED_SET_RR) {
        s->rr = tot;
    } else if (op == RED_STEP_END) {
        end_body(s, tot);
    } else if (op == RED_CHEB_END) {
        end_body(s, tot);
        // Algorithm 3: alpha, beta of the next body
        const double al = 1.0 / (s->cheb_delta + s->beta / s->alpha);
        s->alpha = al;
        s->beta = -(s->cheb_c * al * 0.5) * (s->cheb_c * al * 0.5);
    }
}

// This thread's share of n partial sums, in index order (thread t sums t, t + blockDim, ...);
// loads are issued eight at a time so that one memory latency covers eight of them.
__device__ __forceinline__ double sum_partials(const double* partials, int n)
{
    double v = 0.0;
    const int bd = (int)blockDim.x;
    int i = threadIdx.x;
    for (; i + 7 * bd < n; i += 8 * bd) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; u++) t[u] = partials[i + u * bd];
#pragma unroll
        for (int u = 0; u < 8; u++) v += t[u];
    }
    for (; i < n; i += bd) v += partials[i];
    return v;
}

// A loop reduction deferred by the last pass of the previous body (Scalars::pend_n partial sums)
// is completed by the first workgroup of the next body's first kernel: the partials were written
// by an earlier kernel, so no fence or counter is needed.  Same summation order and scalar update
// as the separate reduction kernel.  All threads of the workgroup call this.
__device__ __forceinline__ void finish_deferred(Scalars* s, const double* partials, double* red)
{
    const int n = s->pend_n;
    if (n == 0) return;
    const double tot = block_sum(sum_partials(partials, n), red);
    if (threadIdx.x == 0) {
        apply_redop(s, s->pend_op, tot);
        s->pend_n = 0;
    }
}

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

// Component c of a [d][n] vector: a uniform base address, so that a point's access is that base
// plus a 32-bit per-lane offset (no 64-bit address arithmetic per access).
template <typename P>
__device__ __forceinline__ P* comp(P* base, int c, unsigned n)
{
    return base + (size_t)c * n;
}

// Batched point processing: the loads of kU points per thread are all issued before any of them
// is used, so one memory latency covers kU points (a loop with a runtime trip count would wait
// once per point).  The operation and coefficient kind are uniform across the launch, so their
// branches sit outside the unrolled point loops; out-of-range points load from point 0 and are
// discarded.
constexpr int kU = 4;

// Points per thread and chunk for a row length L: one chunk covers a tile of up to 8 rows.
constexpr int ku_for(int L)
{
    const int k = (8 * L + kThreads - 1) / kThreads;
    return k < 2 ? 2 : (k > 8 ? 8 : k);
}

// Stage 0 of the first pass for kU points starting at this thread's index base + threadIdx.x:
// z = A(pt) u with u per FirstOp; writes the real rows Zr[(r D + c) L + i].
template <typename T, int D, int L, int KU, bool IL = false, bool XD = false>
__device__ __forceinline__ void first_stage0_chunk(const FirstArgs<T>& a, int op, const T* tab, T beta, int base,
                                                   int total, int lim, long long pt0, T* Zr)
{
    const unsigned npts = (unsigned)a.g.npts;  // 32-bit offsets: d |grid| < 2^31 here
    unsigned pt[KU];
    bool ok[KU];
#pragma unroll
    for (int u = 0; u < KU; u++) {
        const int idx = base + u * (int)blockDim.x + (int)threadIdx.x;
        ok[u] = idx < lim;
        pt[u] = ok[u] ? (unsigned)(pt0 + idx) : 0u;
    }
    T uu[KU][D];
    if (op == OP_E) {
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) uu[u][c] = T(a.E[c]);
    } else if (op == OP_AP_CG) {
        T rr[KU][D], pp[KU][D];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                rr[u][c] = comp(a.r, c, npts)[pt[u]];
                pp[u][c] = comp(a.p, c, npts)[pt[u]];
            }
        if (XD) {  // the previous body's x += alpha p, with p as it was on entry
            const T al = T(a.sc->alpha);
            T xx[KU][D];
#pragma unroll
            for (int u = 0; u < KU; u++)
#pragma unroll
                for (int c = 0; c < D; c++) xx[u][c] = comp(a.xd, c, npts)[pt[u]];
#pragma unroll
            for (int u = 0; u < KU; u++)
#pragma unroll
                for (int c = 0; c < D; c++)
                    if (ok[u]) comp(a.xd, c, npts)[pt[u]] = fma(al, pp[u][c], xx[u][c]);
        }
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                uu[u][c] = rr[u][c] + beta * pp[u][c];
                if (ok[u]) comp(a.p, c, npts)[pt[u]] = uu[u][c];
            }
    } else {
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) uu[u][c] = comp(a.x, c, npts)[pt[u]];
        if (op == OP_AX) {
#pragma unroll
            for (int u = 0; u < KU; u++)
#pragma unroll
                for (int c = 0; c < D; c++) uu[u][c] += T(a.E[c]);
        }
    }
    T z[KU][D];
    if (op == OP_ID) {
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) z[u][c] = uu[u][c];
    } else if (a.A.kind == AK_PHASE) {
        int ph[KU];
#pragma unroll
        for (int u = 0; u < KU; u++) ph[u] = a.A.phase[pt[u]];
#pragma unroll
        for (int u = 0; u < KU; u++) sym_mul<T, D>(tab + 6 * ph[u], uu[u], z[u]);
    } else if (a.A.kind == AK_ISO) {
        const T* cc = static_cast<const T*>(a.A.coef);
        T co[KU];
#pragma unroll
        for (int u = 0; u < KU; u++) co[u] = cc[pt[u]];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) z[u][c] = co[u] * uu[u][c];
    } else {
        const T* cc = static_cast<const T*>(a.A.coef);
        T co[KU][6];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int q = 0; q < ncoef_of<D>(); q++) co[u][q] = comp(cc, q, npts)[pt[u]];
#pragma unroll
        for (int u = 0; u < KU; u++) sym_mul<T, D>(co[u], uu[u], z[u]);
    }
    if (op == OP_EM) {
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) z[u][c] -= T(a.omega) * uu[u][c];
    }
#pragma unroll
    for (int u = 0; u < KU; u++) {
        const int idx = base + u * (int)blockDim.x + (int)threadIdx.x;
        if (idx < total) {
            const int r = idx / L;
            const int i = idx - r * L;
#pragma unroll
            for (int c = 0; c < D; c++) {
                const int q = r * D + c;
                // IL: real rows 2m, 2m+1 interleaved as the real and imaginary parts of complex row m
                const int at = IL ? ((q >> 1) * L + i) * 2 + (q & 1) : q * L + i;
                Zr[at] = ok[u] ? z[u][c] : T(0);
            }
        }
    }
}

// Epilogue of the last pass for kU points: y from the real rows Zr, the solver update per Epi.
template <typename T, int D, int L, int epi, int KU>
__device__ __forceinline__ double last_epilogue_chunk(const LastArgs<T>& a, const T* tabinv, int base,
                                                      int total, int lim, long long pt0, const T* Zr)
{
    const unsigned npts = (unsigned)a.g.npts;  // 32-bit offsets: d |grid| < 2^31 here
    unsigned pt[KU];
    bool ok[KU];
    T y[KU][D];
#pragma unroll
    for (int u = 0; u < KU; u++) {
        const int idx = base + u * (int)blockDim.x + (int)threadIdx.x;
        ok[u] = idx < lim;
        pt[u] = ok[u] ? (unsigned)(pt0 + idx) : 0u;
        const int ii = ok[u] ? idx : 0;
        const int r = ii / L;
        const int i = ii - r * L;
#pragma unroll
        for (int c = 0; c < D; c++) {
            // real rows 2m, 2m+1 are the real and imaginary parts of packed row m (stride L + 1)
            const int q = r * D + c;
            y[u][c] = Zr[((q >> 1) * (L + 1) + i) * 2 + (q & 1)];
        }
    }
    double acc = 0.0;
    if constexpr (epi == EPI_STORE) {
        const T sg = T(a.sgn);
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                const T v = sg * y[u][c];
                if (ok[u]) {
                    comp(a.y, c, npts)[pt[u]] = v;
                    acc += double(v) * double(v);
                }
            }
    } else if constexpr (epi == EPI_RICH) {
        T xv[KU][D];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) xv[u][c] = comp(a.x, c, npts)[pt[u]];
        const T w = T(-a.omega);
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                const T st = w * y[u][c];
                if (ok[u]) {
                    comp(a.x, c, npts)[pt[u]] = xv[u][c] + st;
                    acc += double(st) * double(st);
                }
            }
    } else if constexpr (epi == EPI_CG) {
        T pv[KU][D];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) pv[u][c] = comp(a.p, c, npts)[pt[u]];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++)
                if (ok[u]) {
                    comp(a.q, c, npts)[pt[u]] = y[u][c];
                    acc += double(y[u][c]) * double(pv[u][c]);
                }
    } else if constexpr (epi == EPI_CHEB) {
        T xv[KU][D], rv[KU][D], pv[KU][D];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                const unsigned o = pt[u];
                xv[u][c] = comp(a.x, c, npts)[o];
                rv[u][c] = comp(a.r, c, npts)[o];
                pv[u][c] = comp(a.p, c, npts)[o];
            }
        const T al = T(a.sc ? a.sc->alpha : a.alpha), be = T(a.sc ? a.sc->beta : a.beta);
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                const T rn = rv[u][c] - al * y[u][c];
                if (ok[u]) {
                    const unsigned o = pt[u];
                    comp(a.r, c, npts)[o] = rn;
                    comp(a.x, c, npts)[o] = xv[u][c] + al * pv[u][c];
                    comp(a.p, c, npts)[o] = rn - be * pv[u][c];
                    acc += double(rn) * double(rn);
                }
            }
    } else {  // EPI_EM
        T xv[KU][D], sv[KU][D];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                const unsigned o = pt[u];
                xv[u][c] = comp(a.x, c, npts)[o];
                sv[u][c] = a.src ? comp(a.src, c, npts)[o] : T(2.0 * a.omega * a.E[c]);
            }
        const T w = T(a.omega);
        T xn[KU][D];
        if (a.A.kind == AK_PHASE) {
            int ph[KU];
#pragma unroll
            for (int u = 0; u < KU; u++) ph[u] = a.A.phase[pt[u]];
#pragma unroll
            for (int u = 0; u < KU; u++) {
                T v[D];
#pragma unroll
                for (int c = 0; c < D; c++) v[c] = a.src ? y[u][c] : y[u][c] + sv[u][c];
                sym_mul<T, D>(tabinv + 6 * ph[u], v, xn[u]);
            }
        } else if (a.A.kind == AK_ISO) {
            const T* cc = static_cast<const T*>(a.A.coef);
            T co[KU];
#pragma unroll
            for (int u = 0; u < KU; u++) co[u] = cc[pt[u]];
#pragma unroll
            for (int u = 0; u < KU; u++)
#pragma unroll
                for (int c = 0; c < D; c++) xn[u][c] = (a.src ? y[u][c] : y[u][c] + sv[u][c]) / (co[u] + w);
        } else {
            const T* cc = static_cast<const T*>(a.A.coef);
            T co[KU][6];
#pragma unroll
            for (int u = 0; u < KU; u++)
#pragma unroll
                for (int q = 0; q < ncoef_of<D>(); q++) co[u][q] = comp(cc, q, npts)[pt[u]];
#pragma unroll
            for (int u = 0; u < KU; u++) {
                T v[D];
#pragma unroll
                for (int c = 0; c < D; c++) v[c] = a.src ? y[u][c] : y[u][c] + sv[u][c];
                sym_shift_solve<T, D>(co[u], w, v, xn[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                T xnew = xn[u][c];
                if (a.src) xnew += sv[u][c];
                const T st = xnew - xv[u][c];
                if (ok[u]) {
                    comp(a.x, c, npts)[pt[u]] = xnew;
                    acc += double(st) * double(st);
                }
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
// Workgroup -> tile mapping.  Workgroups are dispatched round-robin over the 8 XCDs (each with
// its own L2); giving every XCD a contiguous range of tiles keeps neighbouring tiles, which share
// cache lines at their edges, on the same L2.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ long long xcd_tile(long long b, long long nb)
{
    const long long q = nb >> 3, r = nb & 7;
    const long long x = b & 7, slot = b >> 3;
    return x * q + (x < r ? x : r) + slot;
}

// ------------------------------------------------------------------------------------------
// Pass 1 (rows of the last axis), all global accesses whole-row contiguous:
//   stage 0  coalesced loads, z = A(x) op x per point -> LDS (real rows)
//   stage A  two real rows (pencils 2m, 2m+1) packed as one complex row, L2-point DFTs -> Y
//   stage B  L1-point DFTs -> the full complex spectrum X of the packed row (LDS)
//   stage S  split into the two real spectra, A(k) = (X(k) + conj X(L-k)) / 2,
//            B(k) = (X(k) - conj X(L-k)) / 2i, and store k < Hb row by row.
// LDS: twiddles | Y (npairs rows) | Zr reals (2 npairs rows), reused as X (npairs rows).
// ------------------------------------------------------------------------------------------
// Points per lane and chunk of stage 0 of the first pass, per precision and length, from timings
// of the pass alone: a tile of about two whole chunks keeps the most loads in flight.  Otherwise
// FP32 chunks of at most 4 points keep four waves per SIMD at the longer rows.
// kx: the same for CG's first pass with the deferred iterate update (three vectors per point).
template <typename T, int L>
struct FirstTune {
    static constexpr int ku = (sizeof(T) == 4 && ku_for(L) > 4) ? 4 : ku_for(L);
    static constexpr int kx = ku > 2 ? ku / 2 : ku;
};
template <>
struct FirstTune<float, 243> {
    static constexpr int ku = 6, kx = 4;  // kx = 6 is as fast but costs a wave per SIMD in every op
};
template <>
struct FirstTune<double, 243> {
    static constexpr int ku = 6, kx = 6;
};

// Stages A, B and S of the first pass in place on the packed complex rows Zc (row m holds real
// rows 2m and 2m+1 as its real and imaginary parts).  Stage A maps all L1 jobs of one row to lanes
// of one wavefront: the wavefront's lanes read all their inputs before any lane writes (one
// instruction stream), so a row can be transformed in its own storage; rows of different waves
// are disjoint.  Stage B is in place per job (it reads and writes the slots k2 + L2 j).
template <typename T, int D, int L1, int L2, int RS = L1 * L2, typename Args>
__device__ __forceinline__ void first_transform_store_ip(const Args& a, long long row0, const cpx<T>* tw, cpx<T>* Zc)
{
    constexpr int L = L1 * L2;
    constexpr int PPW = 64 / L1;  // rows per wavefront in stage A
    static_assert(PPW >= 1, "a row's stage-A jobs must fit one wavefront");
    const int npairs = (a.rpb * D + 1) / 2;
    const int wid = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int nw = (npairs + PPW - 1) / PPW;
    for (int w = wid; w < nw; w += (int)(blockDim.x >> 6)) {
        const int m = w * PPW + lane / L1;
        const int n1 = lane - (lane / L1) * L1;
        const bool act = lane < PPW * L1 && m < npairs;
        if (act) {
            // every store below depends on every load of this lane, and the lanes share one
            // instruction stream: all reads of the wavefront precede its writes
            cpx<T> sv[L2];
            const cpx<T>* z = Zc + m * RS + n1;
#pragma unroll
            for (int n2 = 0; n2 < L2; n2++) sv[n2] = z[L1 * n2];
            reg_dft<T, L2, false>(sv);
            cpx<T>* y = Zc + m * RS + n1 * L2;
            int t = 0;
#pragma unroll
            for (int k2 = 0; k2 < L2; k2++) {
                y[k2] = k2 ? cmul(sv[k2], tw[t]) : sv[k2];
                t += n1;
                if (t >= L) t -= L;
            }
        }
    }
    lds_barrier();
    for (int job = threadIdx.x; job < npairs * L2; job += blockDim.x) {
        const int m = job / L2;
        const int k2 = job - m * L2;
        cpx<T> sv[L1];
        cpx<T>* y = Zc + m * RS + k2;
#pragma unroll
        for (int n1 = 0; n1 < L1; n1++) sv[n1] = y[n1 * L2];
        reg_dft<T, L1, false>(sv);
#pragma unroll
        for (int k1 = 0; k1 < L1; k1++) y[L2 * k1] = sv[k1];
    }
    lds_barrier();
    // stage S: thread (tq, k) stores frequency k of the real rows q = tq, tq + qstep, ...
    // (32-bit element offsets: the plan keeps d |spectrum| below 2^31 for these kernels)
    const int Hb = a.g.Hb;
    const int qstep = (int)blockDim.x / Hb;
    const int tq = (int)threadIdx.x / Hb;
    const int k = (int)threadIdx.x - tq * Hb;
    const int nrows = (int)(a.g.rows - row0 < a.rpb ? a.g.rows - row0 : a.rpb);
    const int qend = nrows * D;
    const unsigned s1 = (unsigned)a.g.s1;
    cpx<T>* outb = a.out + row0 * Hb;  // uniform base, 32-bit per-lane offsets
    if (tq < qstep)
        for (int q = tq; q < qend; q += qstep) {
            const int r = q / D;
            const int c = q - r * D;
            const cpx<T>* x = Zc + (q >> 1) * RS;
            const cpx<T> Z = x[k];
            const cpx<T> Zm = x[k ? L - k : 0];
            const cpx<T> v = (q & 1) ? cpx<T>{T(0.5) * (Z.y + Zm.y), T(-0.5) * (Z.x - Zm.x)}
                                     : cpx<T>{T(0.5) * (Z.x + Zm.x), T(0.5) * (Z.y - Zm.y)};
            outb[(unsigned)c * s1 + (unsigned)(r * Hb + k)] = v;
        }
}

// First pass with one LDS buffer of npairs packed rows (the stages run in place).
// LDS: twiddles | Zc (npairs complex rows) | phase table.
template <typename T, int D, int L1, int L2, int KU = FirstTune<T, L1 * L2>::ku, int KX = FirstTune<T, L1 * L2>::kx>
__device__ __forceinline__ void first_body(const FirstArgs<T>& a, int op, long long b, long long nb)
{
    if (a.done && *a.done) return;
    constexpr int L = L1 * L2;
    extern __shared__ __align__(16) unsigned char smem[];
    const int npairs = (a.rpb * D + 1) / 2;
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* Zc = tw + L;
    T* tab = reinterpret_cast<T*>(Zc + npairs * L);
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    if (a.A.kind == AK_PHASE)
        for (int m = threadIdx.x; m < kMaxPhases * 6; m += blockDim.x) tab[m] = T(a.A.tab[m / 6][m % 6]);
    if ((a.rpb * D) & 1)  // the imaginary half of the last packed row is a zero row
        for (int i = threadIdx.x; i < L; i += blockDim.x) Zc[(npairs - 1) * L + i].y = T(0);
    lds_barrier();
    const long long row0 = xcd_tile(b, nb) * a.rpb;
    const T beta = (op == OP_AP_CG) ? T(a.sc->beta) : T(0);
    {
        const int total = a.rpb * L;
        const long long pt0 = row0 * L;
        const long long left = a.g.rows * (long long)L - pt0;
        const int lim = left < total ? (int)left : total;
        if (op == OP_AP_CG && a.xd) {
            for (int base = 0; base < total; base += KX * blockDim.x)
                first_stage0_chunk<T, D, L, KX, true, true>(a, op, tab, beta, base, total, lim, pt0,
                                                            reinterpret_cast<T*>(Zc));
        } else {
            for (int base = 0; base < total; base += KU * blockDim.x)
                first_stage0_chunk<T, D, L, KU, true>(a, op, tab, beta, base, total, lim, pt0,
                                                      reinterpret_cast<T*>(Zc));
        }
    }
    lds_barrier();
    first_transform_store_ip<T, D, L1, L2>(a, row0, tw, Zc);
}

template <typename T, int D, int L1, int L2>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void k2_first(FirstArgs<T> a, int op)
{
    first_body<T, D, L1, L2>(a, op, blockIdx.x, gridDim.x);
}

// Several plans of one shape in one launch: member blockIdx.y with its own argument block; the
// member's workgroups see the block ids and tile mapping of the single-plan launch.
template <typename T, int D, int L1, int L2>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 8))) void k2_first_b(
    const FirstArgs<T>* __restrict__ tab, int op)
{
    first_body<T, D, L1, L2>(tab[blockIdx.y], op, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------------------------------
// Strided axis pass (3D axis 1), one component per workgroup, tile of P columns.
// ------------------------------------------------------------------------------------------
// b: the workgroup's linear id over the (tile, outer, component) grid gx x gy x gz of one plan.
template <typename T, int L1, int L2, bool INV>
__device__ __forceinline__ void axis_body(const AxisArgs<T>& a, int B, long long b, int gx, int gy, int gz)
{
    if (a.red_sc && b == 0) {
        __shared__ double red[kThreads / 64];
        finish_deferred(a.red_sc, a.partials, red);
    }
    if (a.done && *a.done) return;
    constexpr int L = L1 * L2;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* Y = tw + L;
    const int P = a.P;
    const long long lin = xcd_tile(b, (long long)gx * gy * gz);
    const int tile = (int)(lin % gx);
    const int o = (int)((lin / gx) % gy);
    const int c = (int)(lin / ((long long)gx * gy));
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    lds_barrier();
    const cpx<T>* in = a.in + c * a.in_cs + o * a.in_os;
    cpx<T>* out = a.out + c * a.out_cs + o * a.out_os;
    // a band as long as the axis (GaNi) maps every position to itself: no band test then
    const bool banded = B != L;
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
            if (a.bin && banded) ok = ok && band_index(pos, L, B, &si);
            s[n2] = ok ? in[(unsigned)(si * a.inner + j)] : cpx<T>{T(0), T(0)};
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
    lds_barrier();
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
                if (a.bout && banded && !band_index(pos, L, B, &so)) continue;
                out[(unsigned)(so * a.inner + j)] = s[k1];
            }
        }
    }
}

template <typename T, int L1, int L2, bool INV>
__global__ __launch_bounds__(kThreads) void k2_axis(AxisArgs<T> a, int B)
{
    axis_body<T, L1, L2, INV>(a, B, blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z),
                              gridDim.x, gridDim.y, gridDim.z);
}

// Several plans of one shape: grid (tiles, outer, d x members), member blockIdx.z / d.
template <typename T, int L1, int L2, bool INV>
__global__ __launch_bounds__(kThreads) void k2_axis_b(const AxisArgs<T>* __restrict__ tab, int B, int d)
{
    const int m = (int)blockIdx.z / d;
    const int cz = (int)blockIdx.z - m * d;
    axis_body<T, L1, L2, INV>(tab[m], B, blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * cz),
                              gridDim.x, gridDim.y, d);
}

// ------------------------------------------------------------------------------------------
// Middle pass along axis 0 (all components, in place): forward step A -> LDS -> forward step B,
// multiplier and inverse step B in registers -> LDS -> inverse step A.
// ------------------------------------------------------------------------------------------
template <typename T, int D, int L1, int L2, int MULT>
__device__ __forceinline__ void middle_body(const MidArgs<T>& a, long long b, long long nb)
{
    if (a.done && *a.done) return;
    constexpr int L = L1 * L2;
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* Y = tw + L;
    const int P = a.P;
    const int YS = a.ys;      // LDS stride of a column (L, or L + 1 to spread the banks)
    const int PL = P * YS;
    const int tile = (int)xcd_tile(b, nb);
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    lds_barrier();
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
            s[n2] = (j < a.cols) ? in[(unsigned)((n1 + L1 * n2) * a.cols)] : cpx<T>{T(0), T(0)};
        reg_dft<T, L2, false>(s);
        cpx<T>* y = Y + c * PL + p * YS + n1 * L2;
        int m = 0;
#pragma unroll
        for (int k2 = 0; k2 < L2; k2++) {
            y[k2] = k2 ? cmul(s[k2], tw[m]) : s[k2];
            m += n1;
            if (m >= L) m -= L;
        }
    }
    lds_barrier();
    // forward step B, multiplier, inverse step B: jobs (k2, p)
    const T scale = T(a.scale);
    for (int job = threadIdx.x; job < P * L2; job += blockDim.x) {
        const int k2 = job / P;
        const int p = job - k2 * P;
        const int j = tile * P + p;
        int kv1 = 0, kv2 = 0;
        if (D == 2) {
            kv1 = j;
        } else {
            const int kb1 = j / a.Hb;
            kv1 = signed_index(kb1, a.B1);
            kv2 = j - kb1 * a.Hb;
        }
        const bool colok = j < a.cols;
        // |k|^2 is an integer below 2^24 at these lengths, exact in T
        const T kperp = T(kv1 * kv1 + kv2 * kv2);
        if constexpr (MULT == MULT_G) {
            // G^ is rank one per frequency, (G^ z)_c = k_c t with t = k.z / |k|^2, and along this
            // column only k_0 varies: the components c >= 1 enter through sum_c k_c z_c on the way
            // in and leave as k_c times one inverse transform of t.  Two forward and two inverse
            // L1-point DFTs instead of D of each.
            cpx<T> z0[L1], zp[L1];
            {
                const cpx<T>* y = Y + p * YS + k2;
#pragma unroll
                for (int n1 = 0; n1 < L1; n1++) z0[n1] = y[n1 * L2];
            }
#pragma unroll
            for (int n1 = 0; n1 < L1; n1++) zp[n1] = {T(0), T(0)};
#pragma unroll
            for (int c = 1; c < D; c++) {
                const T kc = T(c == 1 ? kv1 : kv2);
                const cpx<T>* y = Y + c * PL + p * YS + k2;
#pragma unroll
                for (int n1 = 0; n1 < L1; n1++) zp[n1] = zp[n1] + kc * y[n1 * L2];
            }
            reg_dft<T, L1, false>(z0);
            reg_dft<T, L1, false>(zp);
#pragma unroll
            for (int k1 = 0; k1 < L1; k1++) {
                const int pos = k2 + L2 * k1;
                const int k0 = signed_index(pos, L);
                const bool inband = colok && (2 * (k0 < 0 ? -k0 : k0) < a.B0);
                const T kk = T(k0 * k0) + kperp;
                // w = scale / |k|^2, and 0 at k = 0 (G^ vanishes there) and outside the band (Ga)
                const T w = (inband && kk > T(0)) ? scale * recip_int(kk) : T(0);
                const cpx<T> t = w * (T(k0) * z0[k1] + zp[k1]);
                zp[k1] = t;
                z0[k1] = T(k0) * t;
            }
            reg_dft<T, L1, true>(z0);
            reg_dft<T, L1, true>(zp);
            cpx<T>* y = Y + p * YS + k2;
            int m = 0;
#pragma unroll
            for (int n1 = 0; n1 < L1; n1++) {
                const cpx<T> tw_n = conj(tw[m]);
                const cpx<T> v0 = n1 ? cmul(z0[n1], tw_n) : z0[n1];
                const cpx<T> vt = n1 ? cmul(zp[n1], tw_n) : zp[n1];
                y[n1 * L2] = v0;
                y[PL + n1 * L2] = T(kv1) * vt;
                if (D == 3) y[2 * PL + n1 * L2] = T(kv2) * vt;
                m += k2;
                if (m >= L) m -= L;
            }
        } else {
            cpx<T> s[D][L1];
#pragma unroll
            for (int c = 0; c < D; c++) {
                const cpx<T>* y = Y + c * PL + p * YS + k2;
#pragma unroll
                for (int n1 = 0; n1 < L1; n1++) s[c][n1] = y[n1 * L2];
                reg_dft<T, L1, false>(s[c]);
            }
#pragma unroll
            for (int k1 = 0; k1 < L1; k1++) {
                const int pos = k2 + L2 * k1;
                const int k0 = signed_index(pos, L);
                const bool inband = colok && (2 * (k0 < 0 ? -k0 : k0) < a.B0);
                const T kk = T(k0 * k0) + kperp;
                // w = scale / |k|^2, and 0 at k = 0 (I - 2G^ is the identity there); Eyre-Milton
                // runs on the GaNi grid only, where every k is in the band
                const T w = (inband && kk > T(0)) ? scale * recip_int(kk) : T(0);
                const T kvec[3] = {T(k0), T(kv1), T(kv2)};
                cpx<T> kz = {T(0), T(0)};
#pragma unroll
                for (int c = 0; c < D; c++) kz = kz + kvec[c] * s[c][k1];
                const cpx<T> wkz = w * kz;
#pragma unroll
                for (int c = 0; c < D; c++) s[c][k1] = scale * s[c][k1] - T(2) * (kvec[c] * wkz);
            }
#pragma unroll
            for (int c = 0; c < D; c++) {
                reg_dft<T, L1, true>(s[c]);
                cpx<T>* y = Y + c * PL + p * YS + k2;
                int m = 0;
#pragma unroll
                for (int n1 = 0; n1 < L1; n1++) {
                    y[n1 * L2] = n1 ? cmul(s[c][n1], conj(tw[m])) : s[c][n1];
                    m += k2;
                    if (m >= L) m -= L;
                }
            }
        }
    }
    lds_barrier();
    // inverse step A: jobs (c, n1, p)
    for (int job = threadIdx.x; job < D * P * L1; job += blockDim.x) {
        const int cn = job / P;
        const int p = job - cn * P;
        const int c = cn / L1;
        const int n1 = cn - c * L1;
        const int j = tile * P + p;
        cpx<T> s[L2];
        const cpx<T>* y = Y + c * PL + p * YS + n1 * L2;
#pragma unroll
        for (int k2 = 0; k2 < L2; k2++) s[k2] = y[k2];
        reg_dft<T, L2, true>(s);
        if (j < a.cols) {
            cpx<T>* outp = a.buf + c * a.cs + j;
#pragma unroll
            for (int n2 = 0; n2 < L2; n2++) outp[(unsigned)((n1 + L1 * n2) * a.cols)] = s[n2];
        }
    }
}

template <typename T, int D, int L1, int L2, int MULT>
__global__ __launch_bounds__(kThreads) void k2_middle(MidArgs<T> a)
{
    middle_body<T, D, L1, L2, MULT>(a, blockIdx.x, gridDim.x);
}

template <typename T, int D, int L1, int L2, int MULT>
__global__ __launch_bounds__(kThreads) void k2_middle_b(const MidArgs<T>* __restrict__ tab)
{
    middle_body<T, D, L1, L2, MULT>(tab[blockIdx.y], blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------------------------------
// Last pass, all global accesses whole-row contiguous:
//   stage L   coalesced loads of the half spectra of the rows -> LDS (Sx)
//   stage B'  packed row Z = A + iB of pencils 2m, 2m+1 with Hermitian completion
//             (A(L-k) = conj A(k)), inverse L1-point DFTs -> Y
//   stage A'  inverse L2-point DFTs; real and imaginary parts are the two real rows (Zr)
//   stage E   solver epilogue per point, the d components together.
// LDS: twiddles | npairs packed rows of L + 1 slots (half spectra in, real rows out) | table.
// ------------------------------------------------------------------------------------------
// Stages B' and A' of the last pass in place.  Packed row m has its own region of L + 1 complex
// slots: it enters holding the half spectra of real rows 2m and 2m+1 (slots [0, Hb) and
// [Hb, 2Hb)) and leaves holding the two real rows interleaved as one complex row.  Both stages
// map the jobs of one row to lanes of one wavefront, whose lanes read all their inputs before any
// lane writes (one instruction stream); rows of different waves are disjoint.  The caller has
// synchronised after filling S; returns synchronised.
template <typename T, int D, int L1, int L2>
__device__ __forceinline__ void last_transform(const LastArgs<T>& a, const cpx<T>* tw, cpx<T>* S)
{
    constexpr int L = L1 * L2;
    constexpr int LP = L + 1;
    constexpr int PB = 64 / L2, PA = 64 / L1;  // rows per wavefront in stages B' and A'
    static_assert(PB >= 1 && PA >= 1, "a row's jobs must fit one wavefront");
    const int npairs = (a.rpb * D + 1) / 2;
    const int Hb = a.g.Hb;
    const int wid = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63, nwaves = (int)(blockDim.x >> 6);
    for (int w = wid; w < (npairs + PB - 1) / PB; w += nwaves) {
        const int m = w * PB + lane / L2;
        const int k2 = lane - (lane / L2) * L2;
        if (lane < PB * L2 && m < npairs) {
            const cpx<T>* s0 = S + m * LP;
            const cpx<T>* s1 = s0 + Hb;
            cpx<T> sv[L1];
#pragma unroll
            for (int k1 = 0; k1 < L1; k1++) {
                const int k = k2 + L2 * k1;
                cpx<T> A = {T(0), T(0)}, B = {T(0), T(0)};
                if (k < Hb) {
                    A = s0[k];
                    B = s1[k];
                } else if (L - k < Hb) {
                    A = conj(s0[L - k]);
                    B = conj(s1[L - k]);
                }
                sv[k1] = {A.x - B.y, A.y + B.x};
            }
            reg_dft<T, L1, true>(sv);
            cpx<T>* y = S + m * LP + k2;
            int t = 0;
#pragma unroll
            for (int n1 = 0; n1 < L1; n1++) {
                y[n1 * L2] = n1 ? cmul(sv[n1], conj(tw[t])) : sv[n1];
                t += k2;
                if (t >= L) t -= L;
            }
        }
    }
    lds_barrier();
    for (int w = wid; w < (npairs + PA - 1) / PA; w += nwaves) {
        const int m = w * PA + lane / L1;
        const int n1 = lane - (lane / L1) * L1;
        if (lane < PA * L1 && m < npairs) {
            cpx<T> sv[L2];
            cpx<T>* y = S + m * LP;
#pragma unroll
            for (int k2 = 0; k2 < L2; k2++) sv[k2] = y[n1 * L2 + k2];
            reg_dft<T, L2, true>(sv);
#pragma unroll
            for (int n2 = 0; n2 < L2; n2++) y[n1 + L1 * n2] = sv[n2];
        }
    }
    lds_barrier();
}

// Epilogue of the last pass over the tile of rows starting at row0; returns this thread's sum.
template <typename T, int D, int L, int epi, int KUH = 2>  // KUH: points per chunk of the heavy epilogues
__device__ __forceinline__ double last_epilogue_tile(const LastArgs<T>& a, const T* tab, long long row0, const T* Zr)
{
    double acc = 0.0;
    const int total = a.rpb * L;
    const long long pt0 = row0 * L;
    const long long left = a.g.rows * (long long)L - pt0;
    const int lim = left < total ? (int)left : total;
    // the Chebyshev and Eyre-Milton epilogues hold three more vectors per point: smaller chunks
    constexpr int KU = (epi == EPI_CHEB || epi == EPI_EM) && ku_for(L) > KUH ? KUH : ku_for(L);
    for (int base = 0; base < total; base += KU * blockDim.x)
        acc += last_epilogue_chunk<T, D, L, epi, KU>(a, tab, base, total, lim, pt0, Zr);
    return acc;
}

template <typename T, int D, int L1, int L2, int epi>
__device__ __forceinline__ void last_body(const LastArgs<T>& a, int b, int nb)
{
    if (a.done && *a.done) return;
    constexpr int L = L1 * L2;
    extern __shared__ __align__(16) unsigned char smem[];
    const int npairs = (a.rpb * D + 1) / 2;
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* Sx = tw + L;  // npairs packed rows of L + 1 slots
    const T* Zr = reinterpret_cast<const T*>(Sx);
    T* tab = reinterpret_cast<T*>(Sx + npairs * (L + 1));
    __shared__ double red[kThreads / 64];
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    if (epi == EPI_EM && a.A.kind == AK_PHASE)
        for (int m = threadIdx.x; m < kMaxPhases * 6; m += blockDim.x) tab[m] = T(a.A.tab_inv[m / 6][m % 6]);
    const long long row0 = xcd_tile(b, nb) * a.rpb;
    const int Hb = a.g.Hb;
    {
        // stage L: thread (tq, k) loads frequency k of the real rows q = tq, tq + qstep, ...,
        // kQ rows per batch with all loads issued before the LDS stores (32-bit offsets)
        constexpr int kQ = 6;
        const int qstep = (int)blockDim.x / Hb;
        const int tq = (int)threadIdx.x / Hb;
        const int k = (int)threadIdx.x - tq * Hb;
        const int nrows = (int)(a.g.rows - row0 < a.rpb ? a.g.rows - row0 : a.rpb);
        const int qend = nrows * D;
        const unsigned s1 = (unsigned)a.g.s1;
        const cpx<T>* inb = a.in + row0 * Hb;  // uniform base, 32-bit per-lane offsets
        if (tq < qstep)
            for (int q0 = tq; q0 < 2 * npairs; q0 += kQ * qstep) {
                cpx<T> v[kQ];
#pragma unroll
                for (int u = 0; u < kQ; u++) {
                    const int q = q0 + u * qstep;
                    const int r = q / D;
                    const int c = q - r * D;
                    const bool ok = q < qend;
                    const unsigned off = ok ? (unsigned)c * s1 + (unsigned)(r * Hb + k) : (unsigned)k;
                    v[u] = inb[off];
                    if (!ok) v[u] = {T(0), T(0)};
                }
#pragma unroll
                for (int u = 0; u < kQ; u++) {
                    const int q = q0 + u * qstep;
                    if (q < 2 * npairs) Sx[(q >> 1) * (L + 1) + (q & 1) * Hb + k] = v[u];
                }
            }
    }
    lds_barrier();
    last_transform<T, D, L1, L2>(a, tw, Sx);
    const double acc = last_epilogue_tile<T, D, L, epi>(a, tab, row0, Zr);
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) a.partials[b] = tot;
    if (a.defer_sc && b == 0 && threadIdx.x == 0) {
        a.defer_sc->pend_n = nb;
        a.defer_sc->pend_op = a.redop;
    }
}

template <typename T, int D, int L1, int L2, int epi>
__global__ __launch_bounds__(kThreads) void k2_last(LastArgs<T> a)
{
    last_body<T, D, L1, L2, epi>(a, blockIdx.x, gridDim.x);
}

template <typename T, int D, int L1, int L2, int epi>
__global__ __launch_bounds__(kThreads) void k2_last_b(const LastArgs<T>* __restrict__ tab)
{
    last_body<T, D, L1, L2, epi>(tab[blockIdx.y], blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------------------------------
// Last pass of one loop body fused with the first pass of the next (Richardson, Chebyshev,
// Eyre-Milton).  Their updates are pointwise with scalars known before the pass, so once a
// point's iterate is updated the next operator application's operand is known there too:
//   Richardson   x' = x - w y,                   next z = A (x' + E)
//   Chebyshev    r' = r - a y, x' = x + a p,      next z = A p',  p' = r' - b p
//   Eyre-Milton  x' = (A + wI)^{-1} (y + src),    next z = (A - wI) x'
// The tile of rows is inverse-transformed as in the last pass; each point's update and its next
// z are computed by one thread, which writes z into the very LDS slot its y came from; the rows
// are then forward-transformed in place (row stride L + 1) and stored as the next body's first
// spectrum.  This saves the next first pass's read of the iterate and one launch per body.
// ------------------------------------------------------------------------------------------
template <typename T, int D, int L, int epi, int KU>
__device__ __forceinline__ double lastfirst_chunk(const LastArgs<T>& a, const T* tab, const T* tabinv, int base,
                                                  int total, int lim, long long pt0, T* Zr)
{
    const unsigned npts = (unsigned)a.g.npts;  // 32-bit offsets: d |grid| < 2^31 here
    unsigned pt[KU];
    bool ok[KU];
    int at[KU];  // the point's position within its row
    T y[KU][D];
#pragma unroll
    for (int u = 0; u < KU; u++) {
        const int idx = base + u * (int)blockDim.x + (int)threadIdx.x;
        ok[u] = idx < lim;
        pt[u] = ok[u] ? (unsigned)(pt0 + idx) : 0u;
        const int r = idx / L;
        const int i = idx - r * L;
        at[u] = i;
#pragma unroll
        for (int c = 0; c < D; c++) {
            const int q = r * D + c;
            y[u][c] = ok[u] ? Zr[((q >> 1) * (L + 1) + i) * 2 + (q & 1)] : T(0);
        }
    }
    T un[KU][D];
    double acc = 0.0;
    if constexpr (epi == EPI_RICH) {
        T xv[KU][D];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) xv[u][c] = comp(a.x, c, npts)[pt[u]];
        const T w = T(-a.omega);
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                const T st = w * y[u][c];
                const T xn = xv[u][c] + st;
                un[u][c] = xn + T(a.E[c]);
                if (ok[u]) {
                    comp(a.x, c, npts)[pt[u]] = xn;
                    acc += double(st) * double(st);
                }
            }
    } else if constexpr (epi == EPI_CHEB) {
        T xv[KU][D], rv[KU][D], pv[KU][D];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                const unsigned o = pt[u];
                xv[u][c] = comp(a.x, c, npts)[o];
                rv[u][c] = comp(a.r, c, npts)[o];
                pv[u][c] = comp(a.p, c, npts)[o];
            }
        const T al = T(a.sc ? a.sc->alpha : a.alpha), be = T(a.sc ? a.sc->beta : a.beta);
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                const T rn = rv[u][c] - al * y[u][c];
                const T pn = rn - be * pv[u][c];
                un[u][c] = pn + T(a.E[c]);
                if (ok[u]) {
                    const unsigned o = pt[u];
                    comp(a.r, c, npts)[o] = rn;
                    comp(a.x, c, npts)[o] = xv[u][c] + al * pv[u][c];
                    comp(a.p, c, npts)[o] = pn;
                    acc += double(rn) * double(rn);
                }
            }
    } else {  // EPI_EM
        T xv[KU][D], sv[KU][D];
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                const unsigned o = pt[u];
                xv[u][c] = comp(a.x, c, npts)[o];
                sv[u][c] = a.src ? comp(a.src, c, npts)[o] : T(2.0 * a.omega * a.E[c]);
            }
        const T w = T(a.omega);
#pragma unroll
        for (int u = 0; u < KU; u++) {
            T v[D];
#pragma unroll
            for (int c = 0; c < D; c++) v[c] = a.src ? y[u][c] : y[u][c] + sv[u][c];
            coef_shift_solve_rt<T, D>(a.A, tabinv, w, pt[u], npts, v, un[u]);
        }
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) {
                if (a.src) un[u][c] += sv[u][c];
                const T st = un[u][c] - xv[u][c];
                if (ok[u]) {
                    comp(a.x, c, npts)[pt[u]] = un[u][c];
                    acc += double(st) * double(st);
                }
            }
    }
    // the next body's first pass: z = A u (Richardson, Chebyshev) or (A - w I) u (Eyre-Milton)
    T z[KU][D];
#pragma unroll
    for (int u = 0; u < KU; u++) coef_mul_rt<T, D>(a.A, tab, pt[u], npts, un[u], z[u]);
    if constexpr (epi == EPI_EM) {
#pragma unroll
        for (int u = 0; u < KU; u++)
#pragma unroll
            for (int c = 0; c < D; c++) z[u][c] -= T(a.omega) * un[u][c];
    }
#pragma unroll
    for (int u = 0; u < KU; u++) {
        const int idx = base + u * (int)blockDim.x + (int)threadIdx.x;
        if (idx < total) {
            const int r = idx / L;
#pragma unroll
            for (int c = 0; c < D; c++) {
                const int q = r * D + c;
                Zr[((q >> 1) * (L + 1) + at[u]) * 2 + (q & 1)] = ok[u] ? z[u][c] : T(0);
            }
        }
    }
    return acc;
}

template <typename T, int D, int L1, int L2, int epi>
__device__ __forceinline__ void lastfirst_body(const LastArgs<T>& a, int b, int nb)
{
    static_assert(epi == EPI_RICH || epi == EPI_CHEB || epi == EPI_EM, "pointwise updates only");
    if (a.done && *a.done) return;
    constexpr int L = L1 * L2;
    extern __shared__ __align__(16) unsigned char smem[];
    const int npairs = (a.rpb * D + 1) / 2;
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* Sx = tw + L;  // npairs packed rows of L + 1 slots
    T* Zr = reinterpret_cast<T*>(Sx);
    T* tab = reinterpret_cast<T*>(Sx + npairs * (L + 1));
    T* tabinv = tab + kMaxPhases * 6;
    __shared__ double red[kThreads / 64];
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    if (a.A.kind == AK_PHASE)
        for (int m = threadIdx.x; m < kMaxPhases * 6; m += blockDim.x) {
            tab[m] = T(a.A.tab[m / 6][m % 6]);
            tabinv[m] = T(a.A.tab_inv[m / 6][m % 6]);
        }
    const long long row0 = xcd_tile(b, nb) * a.rpb;
    const int Hb = a.g.Hb;
    const int nrows = (int)(a.g.rows - row0 < a.rpb ? a.g.rows - row0 : a.rpb);
    {
        // stage L as in the last pass
        constexpr int kQ = 6;
        const int qstep = (int)blockDim.x / Hb;
        const int tq = (int)threadIdx.x / Hb;
        const int k = (int)threadIdx.x - tq * Hb;
        const int qend = nrows * D;
        const unsigned s1 = (unsigned)a.g.s1;
        const cpx<T>* inb = a.in + row0 * Hb;
        if (tq < qstep)
            for (int q0 = tq; q0 < 2 * npairs; q0 += kQ * qstep) {
                cpx<T> v[kQ];
#pragma unroll
                for (int u = 0; u < kQ; u++) {
                    const int q = q0 + u * qstep;
                    const int r = q / D;
                    const int c = q - r * D;
                    const bool ok = q < qend;
                    const unsigned off = ok ? (unsigned)c * s1 + (unsigned)(r * Hb + k) : (unsigned)k;
                    v[u] = inb[off];
                    if (!ok) v[u] = {T(0), T(0)};
                }
#pragma unroll
                for (int u = 0; u < kQ; u++) {
                    const int q = q0 + u * qstep;
                    if (q < 2 * npairs) Sx[(q >> 1) * (L + 1) + (q & 1) * Hb + k] = v[u];
                }
            }
    }
    lds_barrier();
    last_transform<T, D, L1, L2>(a, tw, Sx);
    double acc = 0.0;
    {
        const int total = a.rpb * L;
        const long long pt0 = row0 * L;
        const long long left = a.g.rows * (long long)L - pt0;
        const int lim = left < total ? (int)left : total;
        constexpr int KU = epi == EPI_RICH ? (ku_for(L) > 3 ? 3 : ku_for(L)) : (ku_for(L) > 2 ? 2 : ku_for(L));
        for (int base = 0; base < total; base += KU * blockDim.x)
            acc += lastfirst_chunk<T, D, L, epi, KU>(a, tab, tabinv, base, total, lim, pt0, Zr);
        if ((a.rpb * D) & 1)  // the imaginary half of the last packed row is a zero row
            for (int i = threadIdx.x; i < L; i += blockDim.x) Sx[(npairs - 1) * (L + 1) + i].y = T(0);
    }
    lds_barrier();
    first_transform_store_ip<T, D, L1, L2, L + 1>(a, row0, tw, Sx);
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) a.partials[b] = tot;
    if (a.defer_sc && b == 0 && threadIdx.x == 0) {
        a.defer_sc->pend_n = nb;
        a.defer_sc->pend_op = a.redop;
    }
}

template <typename T, int D, int L1, int L2, int epi>
__global__ __launch_bounds__(kThreads) void k2_lastfirst(LastArgs<T> a)
{
    lastfirst_body<T, D, L1, L2, epi>(a, blockIdx.x, gridDim.x);
}

template <typename T, int D, int L1, int L2, int epi>
__global__ __launch_bounds__(kThreads) void k2_lastfirst_b(const LastArgs<T>* __restrict__ tab)
{
    lastfirst_body<T, D, L1, L2, epi>(tab[blockIdx.y], blockIdx.x, gridDim.x);
}

// Lengths with specialised kernels; their splits L = L1 * L2 (L1 = 5, 7 or 9: the middle pass holds
// d x L1 values per job in registers) are listed with the launches.
constexpr int kV2Lengths[] = {45, 63, 81, 125, 135, 243};

inline bool v2_supported(int L)
{
    for (int v : kV2Lengths)
        if (v == L) return true;
    return false;
}

}  // namespace fgh
