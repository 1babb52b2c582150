// fgh_kernels.hip -- gfx950 kernels of libfgh: the passes of y = G A x (eq:linsys) with the
// solver epilogues of Algorithms 1-4 fused into the last pass, deterministic FP64 reductions,
// and the set-up kernels (double-grid coefficients, spectral bounds).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cstdlib>

#include "fgh_args.hpp"
#include "fgh_launch.hpp"
#include "fgh_v2.hpp"

namespace fgh {

// ------------------------------------------------------------------------------------------
// Pass 1: real rows along the last axis -> half spectra S1.
// ------------------------------------------------------------------------------------------

template <typename T, int D, int AK, int OP>
__global__ __launch_bounds__(kThreads) void k_first(FirstArgs<T> a)
{
    if (a.done && *a.done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = a.ax.L;
    const int npen = a.npen;
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* b0 = tw + L;
    cpx<T>* b1 = b0 + npen * L;
    T* tab = reinterpret_cast<T*>(b1 + npen * L);
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    if (AK == AK_PHASE)
        for (int m = threadIdx.x; m < kMaxPhases * 6; m += blockDim.x) tab[m] = T(a.A.tab[m / 6][m % 6]);
    const long long row0 = (long long)blockIdx.x * a.rpb;
    const long long npts = a.g.npts;
    if ((a.rpb * D) & 1)
        for (int i = threadIdx.x; i < L; i += blockDim.x) b0[(npen - 1) * L + i].y = T(0);
    __syncthreads();
    const T beta = (OP == OP_AP_CG) ? T(a.sc->beta) : T(0);
    for (int idx = threadIdx.x; idx < a.rpb * L; idx += blockDim.x) {
        const int r = idx / L;
        const int i = idx - r * L;
        const long long row = row0 + r;
        T z[D];
        if (row < a.g.rows) {
            const long long pt = row * L + i;
            T u[D];
#pragma unroll
            for (int c = 0; c < D; c++) {
                if (OP == OP_AX)
                    u[c] = a.x[c * npts + pt] + T(a.E[c]);
                else if (OP == OP_E)
                    u[c] = T(a.E[c]);
                else if (OP == OP_AP_CG) {
                    const T po = a.p[c * npts + pt];
                    if (a.xd) a.xd[c * npts + pt] = fma(T(a.sc->alpha), po, a.xd[c * npts + pt]);
                    const T pn = a.r[c * npts + pt] + beta * po;
                    a.p[c * npts + pt] = pn;
                    u[c] = pn;
                } else
                    u[c] = a.x[c * npts + pt];
            }
            if (OP == OP_ID) {
#pragma unroll
                for (int c = 0; c < D; c++) z[c] = u[c];
            } else {
                T co[6];
                load_coef<T, D, AK>(a.A, tab, pt, npts, co);
                mul_A<T, D, AK>(co, u, z);
                if (OP == OP_EM) {
#pragma unroll
                    for (int c = 0; c < D; c++) z[c] -= T(a.omega) * u[c];
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < D; c++) z[c] = T(0);
        }
#pragma unroll
        for (int c = 0; c < D; c++) {
            const int pp = r * D + c;
            if (pp & 1)
                b0[(pp >> 1) * L + i].y = z[c];
            else
                b0[(pp >> 1) * L + i].x = z[c];
        }
    }
    __syncthreads();
    cpx<T>* res = fft_lds<T, false>(b0, b1, a.ax, npen, tw);
    const int Hb = a.g.Hb;
    const int nreal = a.rpb * D;
    for (int idx = threadIdx.x; idx < npen * Hb; idx += blockDim.x) {
        const int pen = idx / Hb;
        const int k = idx - pen * Hb;
        const cpx<T> Z = res[pen * L + k];
        const cpx<T> Zm = res[pen * L + (k ? L - k : 0)];
        const cpx<T> Av = {T(0.5) * (Z.x + Zm.x), T(0.5) * (Z.y - Zm.y)};
        const cpx<T> Bv = {T(0.5) * (Z.y + Zm.y), T(-0.5) * (Z.x - Zm.x)};
#pragma unroll
        for (int half = 0; half < 2; half++) {
            const int pp = 2 * pen + half;
            if (pp < nreal) {
                const int r = pp / D;
                const int c = pp - r * D;
                const long long row = row0 + r;
                if (row < a.g.rows) a.out[c * a.g.s1 + row * Hb + k] = half ? Bv : Av;
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// Strided pass along a middle axis (3D axis 1), one component per workgroup.
// ------------------------------------------------------------------------------------------

template <typename T, bool INV>
__global__ __launch_bounds__(kThreads) void k_axis(AxisArgs<T> a)
{
    if (a.done && *a.done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = a.ax.L;
    const int P = a.P;
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* b0 = tw + L;
    cpx<T>* b1 = b0 + P * L;
    const int tile = blockIdx.x, o = blockIdx.y, c = blockIdx.z;
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    if (a.nin < L)
        for (int m = threadIdx.x; m < P * L; m += blockDim.x) b0[m] = {T(0), T(0)};
    __syncthreads();
    const cpx<T>* in = a.in + c * a.in_cs + o * a.in_os;
    for (int idx = threadIdx.x; idx < a.nin * P; idx += blockDim.x) {
        const int s = idx / P;
        const int col = idx - s * P;
        const int j = tile * P + col;
        const int pos = a.bin ? band_pos(s, a.nin, L) : s;
        cpx<T> v = {T(0), T(0)};
        if (j < a.inner) v = in[(long long)s * a.inner + j];
        b0[col * L + pos] = v;
    }
    __syncthreads();
    cpx<T>* res = fft_lds<T, INV>(b0, b1, a.ax, P, tw);
    cpx<T>* out = a.out + c * a.out_cs + o * a.out_os;
    for (int idx = threadIdx.x; idx < a.nout * P; idx += blockDim.x) {
        const int s = idx / P;
        const int col = idx - s * P;
        const int j = tile * P + col;
        if (j < a.inner) {
            const int pos = a.bout ? band_pos(s, a.nout, L) : s;
            out[(long long)s * a.inner + j] = res[col * L + pos];
        }
    }
}

// ------------------------------------------------------------------------------------------
// Middle pass along axis 0: forward FFT of every component, Fourier multiplier with all d
// components of a frequency at hand (eq:proj / eq:discrete_proj; Algorithm 4's I - 2G^),
// inverse FFT.  Works in place on the spectrum.
// ------------------------------------------------------------------------------------------

template <typename T, int D, int MULT>
__global__ __launch_bounds__(kThreads) void k_middle(MidArgs<T> a)
{
    if (a.done && *a.done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = a.ax.L;
    const int P = a.P;
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* reg = tw + L;
    const int PL = P * L;
    const int tile = blockIdx.x;
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    for (int idx = threadIdx.x; idx < D * PL; idx += blockDim.x) {
        const int c = idx / PL;
        const int rem = idx - c * PL;
        const int i0 = rem / P;
        const int col = rem - i0 * P;
        const int j = tile * P + col;
        cpx<T> v = {T(0), T(0)};
        if (j < a.cols) v = a.buf[c * a.cs + (long long)i0 * a.cols + j];
        reg[c * PL + col * L + i0] = v;
    }
    __syncthreads();
    int where[D];
    int freebuf = D;
#pragma unroll
    for (int c = 0; c < D; c++) where[c] = c;
#pragma unroll
    for (int c = 0; c < D; c++) {
        cpx<T>* res = fft_lds<T, false>(reg + where[c] * PL, reg + freebuf * PL, a.ax, P, tw);
        if (res != reg + where[c] * PL) {
            const int t = where[c];
            where[c] = freebuf;
            freebuf = t;
        }
    }
    const T scale = T(a.scale);
    for (int idx = threadIdx.x; idx < PL; idx += blockDim.x) {
        const int f = idx / P;
        const int col = idx - f * P;
        const int j = tile * P + col;
        const int k0 = signed_index(f, L);
        const bool inband = (2 * (k0 < 0 ? -k0 : k0) < a.B0) && (j < a.cols);
        int kv[3];
        kv[0] = k0;
        if (D == 2) {
            kv[1] = j;
        } else {
            const int kb1 = j / a.Hb;
            kv[1] = signed_index(kb1, a.B1);
            kv[2] = j - kb1 * a.Hb;
        }
        cpx<T> z[D];
#pragma unroll
        for (int c = 0; c < D; c++) z[c] = reg[where[c] * PL + col * L + f];
        cpx<T> w[D];
        double kk = 0.0;
#pragma unroll
        for (int c = 0; c < D; c++) kk += double(kv[c]) * double(kv[c]);
        if (!inband) {
#pragma unroll
            for (int c = 0; c < D; c++) w[c] = {T(0), T(0)};
        } else if (kk == 0.0) {
#pragma unroll
            for (int c = 0; c < D; c++) w[c] = (MULT == MULT_EM) ? scale * z[c] : cpx<T>{T(0), T(0)};
        } else {
            cpx<T> kz = {T(0), T(0)};
#pragma unroll
            for (int c = 0; c < D; c++) kz = kz + T(kv[c]) * z[c];
            const T inv = T(1.0 / kk);
#pragma unroll
            for (int c = 0; c < D; c++) {
                const cpx<T> gz = (T(kv[c]) * inv) * kz;
                w[c] = (MULT == MULT_G) ? scale * gz : scale * (z[c] - T(2) * gz);
            }
        }
#pragma unroll
        for (int c = 0; c < D; c++) reg[where[c] * PL + col * L + f] = w[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < D; c++) {
        cpx<T>* res = fft_lds<T, true>(reg + where[c] * PL, reg + freebuf * PL, a.ax, P, tw);
        if (res != reg + where[c] * PL) {
            const int t = where[c];
            where[c] = freebuf;
            freebuf = t;
        }
    }
    for (int idx = threadIdx.x; idx < D * PL; idx += blockDim.x) {
        const int c = idx / PL;
        const int rem = idx - c * PL;
        const int i0 = rem / P;
        const int col = rem - i0 * P;
        const int j = tile * P + col;
        if (j < a.cols) a.buf[c * a.cs + (long long)i0 * a.cols + j] = reg[where[c] * PL + col * L + i0];
    }
}

// ------------------------------------------------------------------------------------------
// Last pass: half spectra -> real rows, with the solver epilogue (Algorithms 1-4).
// ------------------------------------------------------------------------------------------

template <typename T, int D, int AK, int EPI>
__global__ __launch_bounds__(kThreads) void k_last(LastArgs<T> a)
{
    if (a.done && *a.done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = a.ax.L;
    const int npen = a.npen;
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
    cpx<T>* b0 = tw + L;
    cpx<T>* b1 = b0 + npen * L;
    T* tab = reinterpret_cast<T*>(b1 + npen * L);
    __shared__ double red[kThreads / 64];
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = a.twg[m];
    if (EPI == EPI_EM && AK == AK_PHASE)
        for (int m = threadIdx.x; m < kMaxPhases * 6; m += blockDim.x) tab[m] = T(a.A.tab_inv[m / 6][m % 6]);
    const long long row0 = (long long)blockIdx.x * a.rpb;
    const int Hb = a.g.Hb;
    const int nreal = a.rpb * D;
    for (int idx = threadIdx.x; idx < npen * L; idx += blockDim.x) {
        const int pen = idx / L;
        const int f = idx - pen * L;
        int kk = -1;
        bool mirror = false;
        if (f < Hb) {
            kk = f;
        } else if (L - f < Hb) {
            kk = L - f;
            mirror = true;
        }
        cpx<T> Z = {T(0), T(0)};
        if (kk >= 0) {
            cpx<T> v[2];
#pragma unroll
            for (int half = 0; half < 2; half++) {
                v[half] = {T(0), T(0)};
                const int pp = 2 * pen + half;
                if (pp < nreal) {
                    const int r = pp / D;
                    const int c = pp - r * D;
                    const long long row = row0 + r;
                    if (row < a.g.rows) v[half] = a.in[c * a.g.s1 + row * Hb + kk];
                }
            }
            if (!mirror)
                Z = {v[0].x - v[1].y, v[0].y + v[1].x};
            else
                Z = {v[0].x + v[1].y, -v[0].y + v[1].x};
        }
        b0[pen * L + f] = Z;
    }
    __syncthreads();
    cpx<T>* res = fft_lds<T, true>(b0, b1, a.ax, npen, tw);
    const long long npts = a.g.npts;
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < a.rpb * L; idx += blockDim.x) {
        const int r = idx / L;
        const int i = idx - r * L;
        const long long row = row0 + r;
        if (row >= a.g.rows) continue;
        const long long pt = row * L + i;
        T y[D];
#pragma unroll
        for (int c = 0; c < D; c++) {
            const int pp = r * D + c;
            const cpx<T> v = res[(pp >> 1) * L + i];
            y[c] = (pp & 1) ? v.y : v.x;
        }
        if (EPI == EPI_STORE) {
#pragma unroll
            for (int c = 0; c < D; c++) {
                const T v = T(a.sgn) * y[c];
                a.y[c * npts + pt] = v;
                acc += double(v) * double(v);
            }
        } else if (EPI == EPI_RICH) {
#pragma unroll
            for (int c = 0; c < D; c++) {
                const T s = T(-a.omega) * y[c];
                a.x[c * npts + pt] += s;
                acc += double(s) * double(s);
            }
        } else if (EPI == EPI_CG) {
#pragma unroll
            for (int c = 0; c < D; c++) {
                a.q[c * npts + pt] = y[c];
                acc += double(y[c]) * double(a.p[c * npts + pt]);
            }
        } else if (EPI == EPI_CHEB) {
            const T al = T(a.sc ? a.sc->alpha : a.alpha), be = T(a.sc ? a.sc->beta : a.beta);
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
        } else if (EPI == EPI_EM) {
            const T w = T(a.omega);
            T v[D], xn[D];
            // plain form: x_new = (A + wI)^{-1} (y + 2 w E); correction form (src != NULL):
            // delta_new = (A + wI)^{-1} y + src, src the double-precision defect
#pragma unroll
            for (int c = 0; c < D; c++) v[c] = a.src ? y[c] : y[c] + T(2.0 * a.omega * a.E[c]);
            if (AK == AK_ISO) {
                const T av = static_cast<const T*>(a.A.coef)[pt];
#pragma unroll
                for (int c = 0; c < D; c++) xn[c] = v[c] / (av + w);
            } else if (AK == AK_PHASE) {
                const int ph = a.A.phase[pt];
                sym_mul<T, D>(tab + ph * 6, v, xn);
            } else {
                T co[6];
                const T* cc = static_cast<const T*>(a.A.coef);
#pragma unroll
                for (int q = 0; q < ncoef_of<D>(); q++) co[q] = cc[q * npts + pt];
                sym_shift_solve<T, D>(co, w, v, xn);
            }
            if (a.src) {
#pragma unroll
                for (int c = 0; c < D; c++) xn[c] += a.src[c * npts + pt];
            }
#pragma unroll
            for (int c = 0; c < D; c++) {
                const long long o = c * npts + pt;
                const T s = xn[c] - a.x[o];
                a.x[o] = xn[c];
                acc += double(s) * double(s);
            }
        }
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = tot;
}

// ------------------------------------------------------------------------------------------
// Reductions and vector kernels.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void reduce_body(const double* __restrict__ partials, int n, Scalars* s, int op)
{
    __shared__ double red[kThreads / 64];
    const bool in_loop = op == RED_CG_ALPHA || op == RED_CG_END || op == RED_STEP_END || op == RED_CHEB_END;
    if (in_loop && s->done) return;
    const double tot = block_sum(sum_partials(partials, n), red);
    if (threadIdx.x == 0) apply_redop(s, op, tot);
}

__global__ __launch_bounds__(kThreads) void k_reduce(const double* __restrict__ partials, int n, Scalars* s, int op)
{
    reduce_body(partials, n, s, op);
}

// One loop reduction per member of a batch (workgroup m: member m).
__global__ __launch_bounds__(kThreads) void k_reduce_b(const ReduceArgs* __restrict__ tab, int op)
{
    const ReduceArgs& a = tab[blockIdx.x];
    reduce_body(a.partials, a.n, a.sc, op);
}

// Start a solver loop: m = 0, done = 0 and the loop's constants (no memset: a plain kernel).
__global__ void k_init_loop(Scalars* s, double rr, double alpha, double beta, double thr, double npts, double blowup,
                            double cheb_c, double cheb_delta, int limit)
{
    s->rr = rr;
    s->alpha = alpha;
    s->beta = beta;
    s->thr = thr;
    s->npts = npts;
    s->blowup = blowup;
    s->cheb_c = cheb_c;
    s->cheb_delta = cheb_delta;
    s->done = 0;
    s->m = 0;
    s->limit = limit;
    s->last = 0.0;
    s->pend_n = 0;
}

// Reduce nvals interleaved partial sums [nblocks][nvals] (fixed order).
__global__ __launch_bounds__(kThreads) void k_reduce_multi(const double* __restrict__ partials, int nblocks,
                                                           int nvals, double* out)
{
    __shared__ double red[kThreads / 64];
    for (int q = 0; q < nvals; q++) {
        double v = 0.0;
        for (int i = threadIdx.x; i < nblocks; i += blockDim.x) v += partials[(long long)i * nvals + q];
        const double tot = block_sum(v, red);
        if (threadIdx.x == 0) out[q] = tot;
        __syncthreads();
    }
}

constexpr int kVecBlocks = 1024;

// Streamed access (double precision): non-temporal loads and stores, which mark the lines for
// early eviction.  In double precision one vector of the large grids exceeds the last-level cache
// anyway, and the update runs at about 6.2 TB/s instead of 5.3; in single precision the r it
// writes is read again by the next first pass and is better left in the cache.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* a)
{
    if constexpr (sizeof(T) == 8) return __builtin_nontemporal_load(a);
    else return *a;
}
template <typename T>
__device__ __forceinline__ void st_stream(T v, T* a)
{
    if constexpr (sizeof(T) == 8) __builtin_nontemporal_store(v, a);
    else *a = v;
}

// x += alpha p (UX; otherwise the next body's first pass applies it), r -= alpha q; returns this
// thread's part of (r, r).  U grid-strided points per batch, all loads issued before any use (one
// memory latency per batch); each thread visits its points in increasing order whatever U is, so
// the sums do not depend on it.
template <typename T, bool UX>
__device__ __forceinline__ double cg_update_loop(long long n, T* __restrict__ x, T* __restrict__ r,
                                                 const T* __restrict__ p, const T* __restrict__ q, T alpha,
                                                 unsigned bx, unsigned gx)
{
    constexpr int U = (!UX && sizeof(T) == 8) ? 8 : 4;
    double acc = 0.0;
    const long long stride = (long long)gx * blockDim.x;
    long long i = (long long)bx * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        T xv[U], pv[U], rv[U], qv[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const long long j = i + u * stride;
            if (UX) {
                xv[u] = ld_stream(x + j);
                pv[u] = ld_stream(p + j);
            }
            rv[u] = ld_stream(r + j);
            qv[u] = ld_stream(q + j);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const long long j = i + u * stride;
            if (UX) st_stream(fma(alpha, pv[u], xv[u]), x + j);
            const T rn = rv[u] - alpha * qv[u];
            st_stream(rn, r + j);
            acc += double(rn) * double(rn);
        }
    }
    for (; i < n; i += stride) {
        if (UX) x[i] = fma(alpha, p[i], x[i]);
        const T rv = r[i] - alpha * q[i];
        r[i] = rv;
        acc += double(rv) * double(rv);
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ void cg_update_body(long long n, T* __restrict__ x, T* __restrict__ r,
                                               const T* __restrict__ p, const T* __restrict__ q, const Scalars* s,
                                               double* partials, unsigned bx, unsigned gx)
{
    __shared__ double red[kThreads / 64];
    if (s->done) return;
    const T alpha = T(s->alpha);
    const double acc = x ? cg_update_loop<T, true>(n, x, r, p, q, alpha, bx, gx)
                         : cg_update_loop<T, false>(n, x, r, p, q, alpha, bx, gx);
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partials[bx] = tot;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_update(long long n, T* __restrict__ x, T* __restrict__ r,
                                                        const T* __restrict__ p, const T* __restrict__ q,
                                                        const Scalars* s, double* partials)
{
    cg_update_body<T>(n, x, r, p, q, s, partials, blockIdx.x, gridDim.x);
}

// The CG update of every member of a batch: grid (kVecBlocks, members).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_update_b(const UpdateArgs<T>* __restrict__ tab)
{
    const UpdateArgs<T>& a = tab[blockIdx.y];
    cg_update_body<T>(a.n, a.x, a.r, a.p, a.q, a.sc, a.partials, blockIdx.x, gridDim.x);
}

// x += alpha p with the loop's last alpha: the update of a CG loop's final body, which the loop
// leaves to the first pass of a body that does not run.  Not gated by the stop flag.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_x(long long n, T* __restrict__ x, const T* __restrict__ p,
                                                   const Scalars* s)
{
    const T alpha = T(s->alpha);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] = fma(alpha, p[i], x[i]);
}

template <typename T>
__global__ void k_fill(long long n, T* x, T v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

template <typename T>
__global__ void k_fill_field(int d, long long npts, T* x, double v0, double v1, double v2)
{
    const double vv[3] = {v0, v1, v2};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < d * npts; i += (long long)gridDim.x * blockDim.x)
        x[i] = T(vv[i / npts]);
}

template <typename T>
__global__ void k_copy(long long n, T* __restrict__ dst, const T* __restrict__ src)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_f64_to_f32(long long n, float* __restrict__ dst, const double* __restrict__ src)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = float(src[i]);
}

__global__ void k_add_f32_to_f64(long long n, double* __restrict__ x, const float* __restrict__ d)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] += double(d[i]);
}

// y = a x + b y
__global__ void k_axpby(long long n, double* __restrict__ y, double a, const double* __restrict__ x, double b)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

__global__ void k_add_f64(long long n, double* __restrict__ x, const double* __restrict__ d)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] += d[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot(long long n, const T* __restrict__ a, const T* __restrict__ b,
                                                  double* partials)
{
    __shared__ double red[kThreads / 64];
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        acc += double(a[i]) * double(b[i]);
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// ||A E||^2 summed over the grid (the scale of the zero right-hand-side test).
template <int D, int AK>
__global__ __launch_bounds__(kThreads) void k_norm_AE(long long npts, CoefArgs A, double E0, double E1, double E2,
                                                      double* partials)
{
    __shared__ double red[kThreads / 64];
    __shared__ double tab[kMaxPhases * 6];
    if (AK == AK_PHASE)
        for (int m = threadIdx.x; m < kMaxPhases * 6; m += blockDim.x) tab[m] = A.tab[m / 6][m % 6];
    __syncthreads();
    const double E[3] = {E0, E1, E2};
    double acc = 0.0;
    for (long long pt = (long long)blockIdx.x * blockDim.x + threadIdx.x; pt < npts; pt += (long long)gridDim.x * blockDim.x) {
        double co[6], z[D];
        load_coef<double, D, AK>(A, tab, pt, npts, co);
        mul_A<double, D, AK>(co, E, z);
#pragma unroll
        for (int c = 0; c < D; c++) acc += z[c] * z[c];
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// A_H and flux (eq:ev_bounds): for each load j, u_j = E_j + e_j, z_j = A u_j;
// partials [block][nrhs*nrhs + nrhs*d]: bilinear (z_j . u_i) then flux z_j.
template <int D, int AK>
__global__ __launch_bounds__(kThreads) void k_effective(long long npts, CoefArgs A, int nrhs, const double* Eall,
                                                        const double* __restrict__ e, double* partials)
{
    __shared__ double red[kThreads / 64];
    __shared__ double tab[kMaxPhases * 6];
    if (AK == AK_PHASE)
        for (int m = threadIdx.x; m < kMaxPhases * 6; m += blockDim.x) tab[m] = A.tab[m / 6][m % 6];
    __syncthreads();
    const int nv = nrhs * nrhs + nrhs * D;
    // at most 3 loads: 9 + 9 accumulators
    double acc[18];
    for (int q = 0; q < 18; q++) acc[q] = 0.0;
    for (long long pt = (long long)blockIdx.x * blockDim.x + threadIdx.x; pt < npts; pt += (long long)gridDim.x * blockDim.x) {
        double co[6];
        load_coef<double, D, AK>(A, tab, pt, npts, co);
        double u[3][D], z[3][D];
        for (int j = 0; j < nrhs; j++) {
#pragma unroll
            for (int c = 0; c < D; c++) u[j][c] = Eall[j * D + c] + e[((long long)j * D + c) * npts + pt];
            mul_A<double, D, AK>(co, u[j], z[j]);
        }
        for (int j = 0; j < nrhs; j++) {
            for (int i = 0; i < nrhs; i++) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < D; c++) s += z[j][c] * u[i][c];
                acc[i * nrhs + j] += s;
            }
#pragma unroll
            for (int c = 0; c < D; c++) acc[nrhs * nrhs + j * D + c] += z[j][c];
        }
    }
    for (int q = 0; q < nv; q++) {
        const double tot = block_sum(acc[q], red);
        if (threadIdx.x == 0) partials[(long long)blockIdx.x * nv + q] = tot;
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------
// Set-up kernels.
// ------------------------------------------------------------------------------------------
__global__ void k_to_f32(long long n, float* dst, const double* src)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = float(src[i]);
}

// Closed-form eigenvalues of symmetric 2x2 / 3x3 blocks (3x3: trigonometric method for the
// roots of the characteristic cubic); per-block min and max -> partials [block][2].
template <int D>
__device__ void sym_eigs(const double* a, double* lo, double* hi)
{
    if (D == 2) {
        const double m = 0.5 * (a[0] + a[2]);
        const double h = 0.5 * (a[0] - a[2]);
        const double rad = sqrt(h * h + a[1] * a[1]);
        *lo = m - rad;
        *hi = m + rad;
    } else {
        const double p1 = a[1] * a[1] + a[2] * a[2] + a[4] * a[4];
        const double q = (a[0] + a[3] + a[5]) / 3.0;
        if (p1 == 0.0) {
            *lo = fmin(a[0], fmin(a[3], a[5]));
            *hi = fmax(a[0], fmax(a[3], a[5]));
            return;
        }
        const double p2 = (a[0] - q) * (a[0] - q) + (a[3] - q) * (a[3] - q) + (a[5] - q) * (a[5] - q) + 2.0 * p1;
        const double p = sqrt(p2 / 6.0);
        const double b00 = (a[0] - q) / p, b11 = (a[3] - q) / p, b22 = (a[5] - q) / p;
        const double b01 = a[1] / p, b02 = a[2] / p, b12 = a[4] / p;
        const double detb = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02);
        double rr = 0.5 * detb;
        rr = fmin(1.0, fmax(-1.0, rr));
        const double phi = acos(rr) / 3.0;
        const double e1 = q + 2.0 * p * cos(phi);
        const double e3 = q + 2.0 * p * cos(phi + 2.0943951023931954923);
        *hi = e1;
        *lo = e3;
    }
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_eig_bounds(int kind, const double* coef, long long npts, double* partials)
{
    __shared__ double rlo[kThreads], rhi[kThreads];
    double lo = 1e300, hi = -1e300;
    for (long long pt = (long long)blockIdx.x * blockDim.x + threadIdx.x; pt < npts; pt += (long long)gridDim.x * blockDim.x) {
        double l, h;
        if (kind == AK_ISO) {
            l = h = coef[pt];
        } else {
            double a[6];
            for (int q = 0; q < ncoef_of<D>(); q++) a[q] = coef[q * npts + pt];
            sym_eigs<D>(a, &l, &h);
        }
        if (!(l == l) || !(h == h)) { l = -1e300; h = 1e300; }  // NaN poisons both bounds
        lo = fmin(lo, l);
        hi = fmax(hi, h);
    }
    rlo[threadIdx.x] = lo;
    rhi[threadIdx.x] = hi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            rlo[threadIdx.x] = fmin(rlo[threadIdx.x], rlo[threadIdx.x + s]);
            rhi[threadIdx.x] = fmax(rhi[threadIdx.x], rhi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = rlo[0];
        partials[2 * blockIdx.x + 1] = rhi[0];
    }
}

__global__ __launch_bounds__(kThreads) void k_minmax(const double* partials, int n, double* out)
{
    __shared__ double rlo[kThreads], rhi[kThreads];
    double lo = 1e300, hi = -1e300;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        lo = fmin(lo, partials[2 * i]);
        hi = fmax(hi, partials[2 * i + 1]);
    }
    rlo[threadIdx.x] = lo;
    rhi[threadIdx.x] = hi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            rlo[threadIdx.x] = fmin(rlo[threadIdx.x], rlo[threadIdx.x + s]);
            rhi[threadIdx.x] = fmax(rhi[threadIdx.x], rhi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = rlo[0];
        out[1] = rhi[0];
    }
}

// Which phases occur: block-local OR in LDS, then one atomic OR per block.
__global__ __launch_bounds__(kThreads) void k_phase_mask(const uint8_t* phase, long long npts, unsigned* mask)
{
    __shared__ unsigned m;
    if (threadIdx.x == 0) m = 0u;
    __syncthreads();
    unsigned loc = 0u;
    for (long long pt = (long long)blockIdx.x * blockDim.x + threadIdx.x; pt < npts; pt += (long long)gridDim.x * blockDim.x)
        loc |= (phase[pt] < 32) ? (1u << phase[pt]) : 0x80000000u;
    atomicOr(&m, loc);
    __syncthreads();
    if (threadIdx.x == 0) atomicOr(mask, m);
}

// Ga assembly, step 1: one real coefficient component on the N grid -> complex buffer.
__global__ void k_coef_component(long long n, int kind, const double* coef, int comp, const uint8_t* phase,
                                 double pv0, double pv1, double pv2, double pv3, double pv4, double pv5,
                                 double pv6, double pv7, double pv8, double pv9, double pv10, double pv11,
                                 double pv12, double pv13, double pv14, double pv15, double2* out)
{
    const double pv[16] = {pv0, pv1, pv2, pv3, pv4, pv5, pv6, pv7, pv8, pv9, pv10, pv11, pv12, pv13, pv14, pv15};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        double v;
        if (kind == AK_PHASE)
            v = pv[phase[i] & 15];
        else if (kind == AK_ISO)
            v = coef[i];
        else
            v = coef[comp * n + i];
        out[i] = make_double2(v, 0.0);
    }
}

// Direct DFT along one axis of a complex grid (set-up only): out[.., k, ..] =
// scale * sum_j in[.., j, ..] w^(j k), w = exp(sign 2 pi i / n) from the table.
__global__ void k_dft_axis(const double2* __restrict__ in, double2* __restrict__ out, long long total, int n,
                           long long stride, const double2* __restrict__ tw, int sign, double scale)
{
    for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < total; o += (long long)gridDim.x * blockDim.x) {
        const long long inner = o % stride;
        const long long k = (o / stride) % n;
        const long long outer = o / (stride * n);
        const double2* src = in + outer * n * stride + inner;
        double sr = 0.0, si = 0.0;
        long long m = 0;
        for (int j = 0; j < n; j++) {
            const double2 w = tw[m];
            const double wi = sign < 0 ? w.y : -w.y;
            const double2 v = src[j * stride];
            sr += v.x * w.x - v.y * wi;
            si += v.x * wi + v.y * w.x;
            m += k;
            if (m >= n) m -= n;
        }
        out[o] = make_double2(scale * sr, scale * si);
    }
}

// Ga assembly, step 2: spectrum on the N grid -> exact pixel Fourier coefficients at the
// frequencies of the double grid (periodic extension times the sinc weights).
__global__ void k_ga_extend(const double2* __restrict__ cn, double2* __restrict__ cm, int d, int N0, int N1, int N2,
                            int M0, int M1, int M2, const double* s0, const double* s1, const double* s2)
{
    const long long nM = (long long)M0 * M1 * (d == 3 ? M2 : 1);
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nM; q += (long long)gridDim.x * blockDim.x) {
        int i[3];
        long long t = q;
        if (d == 3) {
            i[2] = t % M2;
            t /= M2;
        }
        i[1] = t % M1;
        i[0] = t / M1;
        const int Ns[3] = {N0, N1, N2}, Ms[3] = {M0, M1, M2};
        const double* sw[3] = {s0, s1, s2};
        double w = 1.0;
        long long src = 0;
        for (int a = 0; a < d; a++) {
            const int nf = signed_index(i[a], Ms[a]);
            const int r = ((nf % Ns[a]) + Ns[a]) % Ns[a];
            src = src * Ns[a] + r;
            w *= sw[a][i[a]];
        }
        const double2 v = cn[src];
        cm[q] = make_double2(w * v.x, w * v.y);
    }
}

// Twiddle table of one axis on the device: tw[m] = exp(-2 pi i m / L) for m in [0, L), the table
// the passes read between their two DFT steps (the plan uploads the same values from the host).
__global__ void k_twiddles(int L, double2* __restrict__ tw)
{
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < L; m += gridDim.x * blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)m / (double)L, &s, &c);
        tw[m] = make_double2(c, -s);
    }
}

__global__ void k_real_part(long long n, const double2* __restrict__ c, double* __restrict__ out)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = c[i].x;
}

// ==========================================================================================
// Host launch wrappers.
// ==========================================================================================
__global__ void k_set_scalar(double* dst, double v) { *dst = v; }

// Allow dynamic LDS above 64 KB for a kernel (gfx950 has 160 KB per compute unit).
static hipError_t allow_lds(const void* fn, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
// The attribute of each kernel only ever rises, so that no attribute call is made while a stream
// is being captured into a graph once the largest size has been seen.  Raising is serialised per
// kernel: the recorded size is stored only after the call has succeeded and only while holding the
// kernel's lock, so concurrent launches from several threads (server workers, plan-time tuning)
// can neither lower the attribute nor record a size the attribute does not allow.
#define LAUNCH_LDS(KERNEL, GRID, LDS, STREAM, ...)                                              \
    do {                                                                                        \
        static std::atomic<size_t> lds_set_{65536};                                            \
        static std::mutex lds_mu_;                                                              \
        if ((LDS) > lds_set_.load(std::memory_order_acquire)) {                                 \
            std::lock_guard<std::mutex> lds_lk_(lds_mu_);                                       \
            if ((LDS) > lds_set_.load(std::memory_order_relaxed)) {                             \
                hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&KERNEL), (LDS));       \
                if (e_ != hipSuccess) return e_;                                                \
                lds_set_.store((LDS), std::memory_order_release);                               \
            }                                                                                   \
        }                                                                                       \
        if (g_pass_events.start) {                                                              \
            const PassEvents pe_ = g_pass_events;                                               \
            g_pass_events = PassEvents{};                                                       \
            hipExtLaunchKernelGGL(KERNEL, GRID, dim3(kThreads), (LDS), (STREAM), pe_.start, pe_.stop, 0, \
                                  __VA_ARGS__);                                                 \
        } else {                                                                                \
            hipLaunchKernelGGL(KERNEL, GRID, dim3(kThreads), (LDS), (STREAM), __VA_ARGS__);      \
        }                                                                                       \
    } while (0)
static inline unsigned grid_for(long long n, int per = kThreads, int cap = 4096)
{
    long long b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

int vec_blocks() { return kVecBlocks; }

hipError_t Profiler::init(hipStream_t s)
{
    stream = s;
    if (!ready) {
        for (int i = 0; i < 2 * kPool; i++) {
            hipError_t e = hipEventCreate(&ev[i]);
            if (e != hipSuccess) return e;
        }
        ready = true;
    }
    used = 0;
    for (int k = 0; k < PK_KINDS; k++) {
        ms[k] = 0.0;
        n[k] = 0;
        dur[k].clear();
    }
    return hipSuccess;
}

void Profiler::destroy()
{
    if (ready)
        for (int i = 0; i < 2 * kPool; i++) (void)hipEventDestroy(ev[i]);
    ready = false;
}

thread_local PassEvents g_pass_events;

hipError_t Profiler::begin(int k)
{
    if (used == kPool) {
        hipError_t e = drain();
        if (e != hipSuccess) return e;
    }
    kind[used] = k;
    g_pass_events = PassEvents{ev[2 * used], ev[2 * used + 1]};
    return hipSuccess;
}

hipError_t Profiler::end()
{
    hipError_t e = hipSuccess;
    if (g_pass_events.start) {  // no launch took the events: record an empty interval
        g_pass_events = PassEvents{};
        if ((e = hipEventRecord(ev[2 * used], stream)) != hipSuccess) return e;
        e = hipEventRecord(ev[2 * used + 1], stream);
    }
    used++;
    return e;
}

hipError_t Profiler::drain()
{
    if (used == 0) return hipSuccess;
    hipError_t e = hipEventSynchronize(ev[2 * used - 1]);
    if (e != hipSuccess) return e;
    for (int i = 0; i < used; i++) {
        float t = 0.0f;
        e = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
        if (e != hipSuccess) return e;
        ms[kind[i]] += t;
        n[kind[i]]++;
        dur[kind[i]].push_back(t);
    }
    used = 0;
    return hipSuccess;
}

void Profiler::working(int k, double* ms_out, long long* n_out) const
{
    std::vector<float> v = dur[k];
    *ms_out = 0.0;
    *n_out = 0;
    if (v.empty()) return;
    std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
    const float cut = 0.3f * v[v.size() / 2];
    for (float t : dur[k])
        if (t >= cut) {
            *ms_out += t;
            (*n_out)++;
        }
}

template <typename T, int D, int AK>
static hipError_t launch_first_ak(const OpPlan& op, const FirstArgs<T>& fa, int opc, unsigned nblk)
{
    const size_t lds = op.lds_first;
    switch (opc) {
        case OP_AX: LAUNCH_LDS((k_first<T, D, AK, OP_AX>), dim3(nblk), lds, op.stream, fa); break;
        case OP_E: LAUNCH_LDS((k_first<T, D, AK, OP_E>), dim3(nblk), lds, op.stream, fa); break;
        case OP_EM: LAUNCH_LDS((k_first<T, D, AK, OP_EM>), dim3(nblk), lds, op.stream, fa); break;
        case OP_ID: LAUNCH_LDS((k_first<T, D, AK, OP_ID>), dim3(nblk), lds, op.stream, fa); break;
        case OP_AP_CG: LAUNCH_LDS((k_first<T, D, AK, OP_AP_CG>), dim3(nblk), lds, op.stream, fa); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int D, int AK>
static hipError_t launch_last_ak(const OpPlan& op, const LastArgs<T>& la, int epi, unsigned nblk)
{
    const size_t lds = op.lds_first;
    switch (epi) {
        case EPI_STORE: LAUNCH_LDS((k_last<T, D, AK, EPI_STORE>), dim3(nblk), lds, op.stream, la); break;
        case EPI_RICH: LAUNCH_LDS((k_last<T, D, AK, EPI_RICH>), dim3(nblk), lds, op.stream, la); break;
        case EPI_CG: LAUNCH_LDS((k_last<T, D, AK, EPI_CG>), dim3(nblk), lds, op.stream, la); break;
        case EPI_CHEB: LAUNCH_LDS((k_last<T, D, AK, EPI_CHEB>), dim3(nblk), lds, op.stream, la); break;
        case EPI_EM: LAUNCH_LDS((k_last<T, D, AK, EPI_EM>), dim3(nblk), lds, op.stream, la); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int D>
static hipError_t launch_first(const OpPlan& op, const FirstArgs<T>& fa, int opc, unsigned nblk)
{
    switch (op.A.kind) {
        case AK_SYM: return launch_first_ak<T, D, AK_SYM>(op, fa, opc, nblk);
        case AK_ISO: return launch_first_ak<T, D, AK_ISO>(op, fa, opc, nblk);
        case AK_PHASE: return launch_first_ak<T, D, AK_PHASE>(op, fa, opc, nblk);
    }
    return hipErrorInvalidValue;
}

template <typename T, int D>
static hipError_t launch_last(const OpPlan& op, const LastArgs<T>& la, int epi, unsigned nblk)
{
    switch (op.A.kind) {
        case AK_SYM: return launch_last_ak<T, D, AK_SYM>(op, la, epi, nblk);
        case AK_ISO: return launch_last_ak<T, D, AK_ISO>(op, la, epi, nblk);
        case AK_PHASE: return launch_last_ak<T, D, AK_PHASE>(op, la, epi, nblk);
    }
    return hipErrorInvalidValue;
}

template <typename T, int D>
static hipError_t launch_middle(const OpPlan& op, const MidArgs<T>& ma, int mult)
{
    const size_t lds = op.lds_mid;
    if (mult == MULT_G)
        LAUNCH_LDS((k_middle<T, D, MULT_G>), dim3(ma.ntiles), lds, op.stream, ma);
    else
        LAUNCH_LDS((k_middle<T, D, MULT_EM>), dim3(ma.ntiles), lds, op.stream, ma);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_axis(const OpPlan& op, const AxisArgs<T>& xa, bool inv, int outer)
{
    dim3 grid(xa.ntiles, outer, op.g.d);
    if (inv)
        LAUNCH_LDS((k_axis<T, true>), grid, op.lds_axis, op.stream, xa);
    else
        LAUNCH_LDS((k_axis<T, false>), grid, op.lds_axis, op.stream, xa);
    return hipGetLastError();
}

// Size-specialised launches: length, L1, L2 (the lengths of kV2Lengths).
#define V2_ROW_CASES(X) X(45, 5, 9) X(63, 7, 9) X(81, 9, 9) X(125, 5, 25) X(135, 9, 15) X(243, 9, 27)
#define V2_COL_CASES(X) X(45, 5, 9) X(63, 7, 9) X(81, 9, 9) X(125, 5, 25) X(135, 9, 15) X(243, 9, 27)

template <typename T, int D>
static hipError_t v2_first(const OpPlan& op, const FirstArgs<T>& fa, int opc, unsigned nblk)
{
    const size_t lds = fa.xd ? op.lds_first_x : op.lds_first_v2;
    switch (fa.ax.L) {
#define C(LL, A1, A2) \
    case LL: LAUNCH_LDS((k2_first<T, D, A1, A2>), dim3(nblk), lds, op.stream, fa, opc); break;
        V2_ROW_CASES(C)
#undef C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// nblk: the tile count, one workgroup (and one partial sum) per tile.
template <typename T, int D, int EPI>
static hipError_t v2_last_epi(const OpPlan& op, const LastArgs<T>& la, unsigned* nblk)
{
    const size_t lds = op.lds_last_v2;
    switch (la.ax.L) {
#define C(LL, A1, A2) \
    case LL: LAUNCH_LDS((k2_last<T, D, A1, A2, EPI>), dim3(*nblk), lds, op.stream, la); break;
        V2_ROW_CASES(C)
#undef C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int D>
static hipError_t v2_last(const OpPlan& op, const LastArgs<T>& la, int epi, unsigned* nblk)
{
    switch (epi) {
        case EPI_STORE: return v2_last_epi<T, D, EPI_STORE>(op, la, nblk);
        case EPI_RICH: return v2_last_epi<T, D, EPI_RICH>(op, la, nblk);
        case EPI_CG: return v2_last_epi<T, D, EPI_CG>(op, la, nblk);
        case EPI_CHEB: return v2_last_epi<T, D, EPI_CHEB>(op, la, nblk);
        case EPI_EM: return v2_last_epi<T, D, EPI_EM>(op, la, nblk);
    }
    return hipErrorInvalidValue;
}

// Fused last + first pass: the last pass's LDS plus a second coefficient table.
template <typename T, int D, int EPI>
static hipError_t v2_lastfirst_epi(const OpPlan& op, const LastArgs<T>& la, unsigned* nblk)
{
    const size_t lds = op.lds_fused;
    switch (la.ax.L) {
#define C(LL, A1, A2) \
    case LL: LAUNCH_LDS((k2_lastfirst<T, D, A1, A2, EPI>), dim3(*nblk), lds, op.stream, la); break;
        V2_ROW_CASES(C)
#undef C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int D>
static hipError_t v2_lastfirst(const OpPlan& op, const LastArgs<T>& la, int epi, unsigned* nblk)
{
    switch (epi) {
        case EPI_RICH: return v2_lastfirst_epi<T, D, EPI_RICH>(op, la, nblk);
        case EPI_CHEB: return v2_lastfirst_epi<T, D, EPI_CHEB>(op, la, nblk);
        case EPI_EM: return v2_lastfirst_epi<T, D, EPI_EM>(op, la, nblk);
    }
    return hipErrorInvalidValue;
}

template <typename T, int D>
static hipError_t v2_middle(const OpPlan& op, const MidArgs<T>& ma, int mult)
{
    const size_t lds = op.lds_mid;
    switch (ma.ax.L) {
#define C(LL, A1, A2)                                                                          \
    case LL:                                                                                   \
        if (mult == MULT_G)                                                                    \
            LAUNCH_LDS((k2_middle<T, D, A1, A2, MULT_G>), dim3(ma.ntiles), lds, op.stream, ma);  \
        else                                                                                   \
            LAUNCH_LDS((k2_middle<T, D, A1, A2, MULT_EM>), dim3(ma.ntiles), lds, op.stream, ma); \
        break;
        V2_COL_CASES(C)
#undef C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t v2_axis(const OpPlan& op, const AxisArgs<T>& xa, bool inv, int outer, int B)
{
    dim3 grid(xa.ntiles, outer, op.g.d);
    const size_t lds = op.lds_axis;
    switch (xa.ax.L) {
#define C(LL, A1, A2)                                                                        \
    case LL:                                                                                 \
        if (inv)                                                                             \
            LAUNCH_LDS((k2_axis<T, A1, A2, true>), grid, lds, op.stream, xa, B);             \
        else                                                                                 \
            LAUNCH_LDS((k2_axis<T, A1, A2, false>), grid, lds, op.stream, xa, B);            \
        break;
        V2_COL_CASES(C)
#undef C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- batched launches (several plans of one shape): grid y (strided pass: z) over the members
template <typename T, int D>
static hipError_t v2_first_b(const OpPlan& op, const FirstArgs<T>* tab, int opc, unsigned nblk, int nb)
{
    const size_t lds = op.lds_first_v2;
    const dim3 grid(nblk, nb);
    switch (op.ax[D - 1].L) {
#define C(LL, A1, A2)                                                                   \
    case LL:                                                                            \
        LAUNCH_LDS((k2_first_b<T, D, A1, A2>), grid, lds, op.stream, tab, opc);         \
        break;
        V2_ROW_CASES(C)
#undef C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int D>
static hipError_t v2_last_b(const OpPlan& op, const LastArgs<T>* tab, int epi, bool fused, unsigned nblk, int nb)
{
    const dim3 grid(nblk, nb);
    // the loops that share launches: CG bodies (last pass with the CG epilogue) and fused
    // Eyre-Milton bodies
    if (!fused && epi == EPI_CG) {
        const size_t lds = op.lds_last_v2;
        switch (op.ax[D - 1].L) {
#define C(LL, A1, A2)                                                                          \
    case LL:                                                                                   \
        LAUNCH_LDS((k2_last_b<T, D, A1, A2, EPI_CG>), grid, lds, op.stream, tab);              \
        break;
            V2_ROW_CASES(C)
#undef C
            default: return hipErrorInvalidValue;
        }
    } else if (fused && epi == EPI_EM) {
        const size_t lds = op.lds_fused;
        switch (op.ax[D - 1].L) {
#define C(LL, A1, A2)                                                                          \
    case LL:                                                                                   \
        LAUNCH_LDS((k2_lastfirst_b<T, D, A1, A2, EPI_EM>), grid, lds, op.stream, tab);         \
        break;
            V2_ROW_CASES(C)
#undef C
            default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int D>
static hipError_t v2_middle_b(const OpPlan& op, const MidArgs<T>* tab, int mult, int ntiles, int nb)
{
    const size_t lds = op.lds_mid;
    const dim3 grid(ntiles, nb);
    switch (op.ax[0].L) {
#define C(LL, A1, A2)                                                                          \
    case LL:                                                                                   \
        if (mult == MULT_G)                                                                    \
            LAUNCH_LDS((k2_middle_b<T, D, A1, A2, MULT_G>), grid, lds, op.stream, tab);        \
        else                                                                                   \
            LAUNCH_LDS((k2_middle_b<T, D, A1, A2, MULT_EM>), grid, lds, op.stream, tab);       \
        break;
        V2_COL_CASES(C)
#undef C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t v2_axis_b(const OpPlan& op, const AxisArgs<T>* tab, bool inv, int ntiles, int outer, int B, int nb)
{
    const dim3 grid(ntiles, outer, op.g.d * nb);
    const size_t lds = op.lds_axis;
    switch (op.ax[1].L) {
#define C(LL, A1, A2)                                                                           \
    case LL:                                                                                    \
        if (inv)                                                                                \
            LAUNCH_LDS((k2_axis_b<T, A1, A2, true>), grid, lds, op.stream, tab, B, op.g.d);     \
        else                                                                                    \
            LAUNCH_LDS((k2_axis_b<T, A1, A2, false>), grid, lds, op.stream, tab, B, op.g.d);    \
        break;
        V2_COL_CASES(C)
#undef C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static MidArgs<T> mid_args(const OpPlan& op, cpx<T>* buf, const int* done)
{
    const Geo& g = op.g;
    MidArgs<T> ma;
    ma.ax = op.ax[0];
    ma.B0 = g.B[0];
    ma.cols = g.cols_mid;
    ma.Hb = g.Hb;
    ma.B1 = g.B[1];
    ma.P = op.P_mid;
    ma.ys = g.L[0] + op.mid_pad;
    ma.ntiles = (g.cols_mid + op.P_mid - 1) / op.P_mid;
    ma.cs = (long long)g.L[0] * g.cols_mid;
    ma.scale = 1.0 / (double)g.npts;
    ma.buf = buf;
    ma.twg = static_cast<const cpx<T>*>(op.tw[0]);
    ma.done = done;
    return ma;
}

// The argument blocks of one application: what the passes read (first pass operator and operand,
// strided and middle geometry, last-pass epilogue), tile counts and flags.
template <typename T, int D>
static hipError_t build_bundle_d(const OpPlan& op, const ApplyArgs& a, ApplyBundle<T>* bu)
{
    const Geo& g = op.g;
    const int last = D - 1;
    cpx<T>* SA = static_cast<cpx<T>*>(op.SA);
    cpx<T>* SB = static_cast<cpx<T>*>(op.SB);
    bu->op = a.op;
    bu->mult = a.mult;
    bu->epi = a.epi;
    bu->skip_first = a.skip_first;
    bu->first_only = a.first_only;

    FirstArgs<T>& fa = bu->fa;
    fa.g = g;
    fa.ax = op.ax[last];
    const int rpb1 = op.v2_row ? (a.x_cg ? op.rpb_first_x : op.rpb_first) : op.rpb;
    bu->nblk1 = (unsigned)((g.rows + rpb1 - 1) / rpb1);
    fa.rpb = rpb1;
    fa.npen = (rpb1 * D + 1) / 2;
    fa.x = static_cast<const T*>(a.x);
    fa.p = static_cast<T*>(a.p_cg);
    fa.r = static_cast<const T*>(a.r_cg);
    fa.xd = static_cast<T*>(a.x_cg);
    fa.sc = op.sc;
    const int* done = a.loop ? &op.sc->done : nullptr;
    fa.done = done;
    for (int c = 0; c < 3; c++) fa.E[c] = a.E[c];
    fa.omega = a.omega;
    fa.A = op.A;
    fa.out = SA;
    fa.twg = static_cast<const cpx<T>*>(op.tw[last]);

    cpx<T>* mid = SA;
    if (D == 3) {
        AxisArgs<T>& xa = bu->xf;
        xa.ax = op.ax[1];
        xa.nin = g.L[1];
        xa.nout = g.B[1];
        xa.bin = 0;
        xa.bout = 1;
        xa.inner = g.Hb;
        xa.P = op.P_axis;
        xa.ntiles = (g.Hb + op.P_axis - 1) / op.P_axis;
        xa.in_os = (long long)g.L[1] * g.Hb;
        xa.out_os = (long long)g.B[1] * g.Hb;
        xa.in_cs = g.s1;
        xa.out_cs = g.s2;
        xa.in = SA;
        xa.out = SB;
        xa.twg = static_cast<const cpx<T>*>(op.tw[1]);
        xa.done = done;
        // the previous body's deferred loop reduction is completed by this pass's first workgroup
        xa.red_sc = a.defer_redop >= 0 ? op.sc : nullptr;
        xa.partials = op.partials;
        mid = SB;
        AxisArgs<T>& xi = bu->xi;
        xi.ax = op.ax[1];
        xi.nin = g.B[1];
        xi.nout = g.L[1];
        xi.bin = 1;
        xi.bout = 0;
        xi.inner = g.Hb;
        xi.P = op.P_axis;
        xi.ntiles = (g.Hb + op.P_axis - 1) / op.P_axis;
        xi.in_os = (long long)g.B[1] * g.Hb;
        xi.out_os = (long long)g.L[1] * g.Hb;
        xi.in_cs = g.s2;
        xi.out_cs = g.s1;
        xi.in = SB;
        xi.out = SA;
        xi.twg = static_cast<const cpx<T>*>(op.tw[1]);
        xi.done = done;
    }
    bu->ma = mid_args<T>(op, mid, done);

    LastArgs<T>& la = bu->la;
    la.g = g;
    la.ax = op.ax[last];
    la.rpb = op.rpb;
    la.npen = op.npen;
    la.in = SA;
    la.y = static_cast<T*>(a.y);
    la.x = static_cast<T*>(a.ex);
    la.r = static_cast<T*>(a.er);
    la.p = static_cast<T*>(a.ep);
    la.q = static_cast<T*>(a.eq);
    la.src = static_cast<const T*>(a.src);
    for (int c = 0; c < 3; c++) la.E[c] = a.E[c];
    la.omega = a.omega;
    la.alpha = a.alpha;
    la.beta = a.beta;
    la.sgn = a.sgn;
    la.A = op.A;
    la.partials = op.partials;
    la.twg = static_cast<const cpx<T>*>(op.tw[last]);
    la.done = done;
    la.sc = a.cheb_dev ? op.sc : nullptr;
    la.out = SA;
    if (a.defer_redop >= 0 && !(D == 3 && op.v2_axis && op.v2_row)) return hipErrorInvalidValue;
    la.defer_sc = a.defer_redop >= 0 ? op.sc : nullptr;
    la.redop = a.defer_redop;
    const bool fused = a.next_op >= 0;
    if (fused && (!fusable(op) || a.next_op != (a.epi == EPI_EM ? OP_EM : OP_AX) ||
                  (a.epi != EPI_RICH && a.epi != EPI_CHEB && a.epi != EPI_EM)))
        return hipErrorInvalidValue;
    bu->fused = fused;
    bu->nblk_last = (unsigned)((g.rows + op.rpb - 1) / op.rpb);
    if (fused) {
        // the fused pass has its own (tuned, even) rows per block
        la.rpb = op.rpb_fused;
        la.npen = (op.rpb_fused * D + 1) / 2;
        bu->nblk_last = (unsigned)((g.rows + op.rpb_fused - 1) / op.rpb_fused);
    }
    return hipSuccess;
}

template <typename T, int D>
static hipError_t apply_d(const OpPlan& op, const ApplyArgs& a, int* nblocks_last)
{
    const Geo& g = op.g;
    ApplyBundle<T> bu{};
    hipError_t e = build_bundle_d<T, D>(op, a, &bu);
    if (e != hipSuccess) return e;
    if (!a.skip_first) {
        const bool prof_PK_FIRST = op.prof && op.prof->wants(PK_FIRST);
        if (prof_PK_FIRST && (e = op.prof->begin(PK_FIRST)) != hipSuccess) return e;
        if ((e = op.v2_row ? v2_first<T, D>(op, bu.fa, a.op, bu.nblk1) : launch_first<T, D>(op, bu.fa, a.op, bu.nblk1)) !=
            hipSuccess)
            return e;
        if (prof_PK_FIRST && (e = op.prof->end()) != hipSuccess) return e;
    }
    if (a.first_only) return hipSuccess;
    if (D == 3) {
        const bool prof_PK_AXIS_FWD = op.prof && op.prof->wants(PK_AXIS_FWD);
        if (prof_PK_AXIS_FWD && (e = op.prof->begin(PK_AXIS_FWD)) != hipSuccess) return e;
        if ((e = op.v2_axis ? v2_axis<T>(op, bu.xf, false, g.L[0], g.B[1]) : launch_axis<T>(op, bu.xf, false, g.L[0])) !=
            hipSuccess)
            return e;
        if (prof_PK_AXIS_FWD && (e = op.prof->end()) != hipSuccess) return e;
    }
    const bool prof_PK_MIDDLE = op.prof && op.prof->wants(PK_MIDDLE);
    if (prof_PK_MIDDLE && (e = op.prof->begin(PK_MIDDLE)) != hipSuccess) return e;
    if ((e = op.v2_mid ? v2_middle<T, D>(op, bu.ma, a.mult) : launch_middle<T, D>(op, bu.ma, a.mult)) != hipSuccess)
        return e;
    if (prof_PK_MIDDLE && (e = op.prof->end()) != hipSuccess) return e;
    if (D == 3) {
        const bool prof_PK_AXIS_INV = op.prof && op.prof->wants(PK_AXIS_INV);
        if (prof_PK_AXIS_INV && (e = op.prof->begin(PK_AXIS_INV)) != hipSuccess) return e;
        if ((e = op.v2_axis ? v2_axis<T>(op, bu.xi, true, g.L[0], g.B[1]) : launch_axis<T>(op, bu.xi, true, g.L[0])) !=
            hipSuccess)
            return e;
        if (prof_PK_AXIS_INV && (e = op.prof->end()) != hipSuccess) return e;
    }
    unsigned nblk = bu.nblk_last;
    const bool prof_PK_LAST = op.prof && op.prof->wants(PK_LAST);
    if (prof_PK_LAST && (e = op.prof->begin(PK_LAST)) != hipSuccess) return e;
    if ((e = bu.fused      ? v2_lastfirst<T, D>(op, bu.la, a.epi, &nblk)
             : op.v2_row ? v2_last<T, D>(op, bu.la, a.epi, &nblk)
                         : launch_last<T, D>(op, bu.la, a.epi, nblk)) != hipSuccess)
        return e;
    if (prof_PK_LAST && (e = op.prof->end()) != hipSuccess) return e;
    if (nblocks_last) *nblocks_last = (int)nblk;
    return hipSuccess;
}

template <typename T>
hipError_t run_middle_only(const OpPlan& op)
{
    cpx<T>* buf = static_cast<cpx<T>*>(op.g.d == 3 ? op.SB : op.SA);
    const MidArgs<T> ma = mid_args<T>(op, buf, nullptr);
    if (op.g.d == 2) return op.v2_mid ? v2_middle<T, 2>(op, ma, MULT_G) : launch_middle<T, 2>(op, ma, MULT_G);
    return op.v2_mid ? v2_middle<T, 3>(op, ma, MULT_G) : launch_middle<T, 3>(op, ma, MULT_G);
}
template hipError_t run_middle_only<double>(const OpPlan&);
template hipError_t run_middle_only<float>(const OpPlan&);

template <typename T>
hipError_t run_axis_only(const OpPlan& op)
{
    const Geo& g = op.g;
    if (g.d != 3) return hipErrorInvalidValue;
    AxisArgs<T> xa{};
    xa.ax = op.ax[1];
    xa.nin = g.L[1];
    xa.nout = g.B[1];
    xa.bin = 0;
    xa.bout = 1;
    xa.inner = g.Hb;
    xa.P = op.P_axis;
    xa.ntiles = (g.Hb + op.P_axis - 1) / op.P_axis;
    xa.in_os = (long long)g.L[1] * g.Hb;
    xa.out_os = (long long)g.B[1] * g.Hb;
    xa.in_cs = g.s1;
    xa.out_cs = g.s2;
    xa.in = static_cast<cpx<T>*>(op.SA);
    xa.out = static_cast<cpx<T>*>(op.SB);
    xa.twg = static_cast<const cpx<T>*>(op.tw[1]);
    xa.done = nullptr;
    return op.v2_axis ? v2_axis<T>(op, xa, false, g.L[0], g.B[1]) : launch_axis<T>(op, xa, false, g.L[0]);
}
template hipError_t run_axis_only<double>(const OpPlan&);
template hipError_t run_axis_only<float>(const OpPlan&);

template <typename T>
hipError_t run_first_only(const OpPlan& op, const T* x)
{
    const Geo& g = op.g;
    const int d = g.d;
    FirstArgs<T> fa{};
    fa.done = nullptr;
    fa.g = g;
    fa.ax = op.ax[d - 1];
    fa.rpb = op.rpb_first;
    fa.npen = (op.rpb_first * d + 1) / 2;
    fa.x = x;
    fa.A = op.A;
    fa.out = static_cast<cpx<T>*>(op.SA);
    fa.twg = static_cast<const cpx<T>*>(op.tw[d - 1]);
    const unsigned nblk = (unsigned)((g.rows + op.rpb_first - 1) / op.rpb_first);
    return d == 2 ? v2_first<T, 2>(op, fa, OP_ID, nblk) : v2_first<T, 3>(op, fa, OP_ID, nblk);
}
template hipError_t run_first_only<double>(const OpPlan&, const double*);
template hipError_t run_first_only<float>(const OpPlan&, const float*);

template <typename T>
hipError_t run_first_cg_only(const OpPlan& op, T* x, const T* r, T* p)
{
    const Geo& g = op.g;
    const int d = g.d;
    FirstArgs<T> fa{};
    fa.done = nullptr;
    fa.g = g;
    fa.ax = op.ax[d - 1];
    fa.rpb = op.rpb_first_x;
    fa.npen = (op.rpb_first_x * d + 1) / 2;
    fa.p = p;
    fa.r = r;
    fa.xd = x;
    fa.sc = op.sc;
    fa.A = op.A;
    fa.out = static_cast<cpx<T>*>(op.SA);
    fa.twg = static_cast<const cpx<T>*>(op.tw[d - 1]);
    const unsigned nblk = (unsigned)((g.rows + op.rpb_first_x - 1) / op.rpb_first_x);
    return d == 2 ? v2_first<T, 2>(op, fa, OP_AP_CG, nblk) : v2_first<T, 3>(op, fa, OP_AP_CG, nblk);
}
template hipError_t run_first_cg_only<double>(const OpPlan&, double*, const double*, double*);
template hipError_t run_first_cg_only<float>(const OpPlan&, float*, const float*, float*);

template <typename T>
hipError_t run_fused_only(const OpPlan& op, T* x)
{
    // the pass multiplies by A: the plan's coefficients must be set
    if (op.A.kind == AK_PHASE ? op.A.phase == nullptr : op.A.coef == nullptr) return hipErrorInvalidValue;
    OpPlan o = op;
    o.prof = nullptr;
    const Geo& g = op.g;
    LastArgs<T> la{};
    la.g = g;
    la.ax = op.ax[g.d - 1];
    la.rpb = op.rpb_fused;
    la.npen = (op.rpb_fused * g.d + 1) / 2;
    la.in = static_cast<const cpx<T>*>(op.SA);
    la.x = x;
    la.omega = 0.0;
    la.sgn = 1.0;
    la.A = op.A;
    la.partials = op.partials;
    la.twg = static_cast<const cpx<T>*>(op.tw[g.d - 1]);
    la.out = static_cast<cpx<T>*>(op.SA);
    unsigned nblk = (unsigned)((g.rows + op.rpb_fused - 1) / op.rpb_fused);
    return g.d == 2 ? v2_lastfirst<T, 2>(o, la, EPI_RICH, &nblk) : v2_lastfirst<T, 3>(o, la, EPI_RICH, &nblk);
}
template hipError_t run_fused_only<double>(const OpPlan&, double*);
template hipError_t run_fused_only<float>(const OpPlan&, float*);

// One strided-axis launch with explicit geometry (generic kernel, any length): transform along
// an axis of length ax.L for `outer` blocks of `inner` contiguous columns per component.
static hipError_t axis_custom(const OpPlan& op, const Axis& ax, const void* tw, bool inv, int nin, int bin, int nout,
                              int bout, int inner, int outer, long long in_os, long long out_os, long long in_cs,
                              long long out_cs, const double2* in, double2* out)
{
    AxisArgs<double> xa{};
    xa.done = nullptr;
    xa.ax = ax;
    xa.nin = nin;
    xa.nout = nout;
    xa.bin = bin;
    xa.bout = bout;
    xa.inner = inner;
    int P = 16;
    while (P > 1 && (size_t)(ax.L + 2 * P * ax.L) * 16 > 80 * 1024) P >>= 1;
    xa.P = P;
    xa.ntiles = (inner + P - 1) / P;
    xa.in_os = in_os;
    xa.out_os = out_os;
    xa.in_cs = in_cs;
    xa.out_cs = out_cs;
    xa.in = reinterpret_cast<const cpx<double>*>(in);
    xa.out = reinterpret_cast<cpx<double>*>(out);
    xa.twg = static_cast<const cpx<double>*>(tw);
    OpPlan o = op;
    o.lds_axis = (size_t)(ax.L + 2 * P * ax.L) * 16;
    return launch_axis<double>(o, xa, inv, outer);
}

hipError_t run_prolong(const OpPlan& opn, const OpPlan& opm, const double* xn, double* ym)
{
    const Geo& gn = opn.g;
    const Geo& gm = opm.g;
    const int d = gn.d;
    hipError_t e;
    double2* A = static_cast<double2*>(opm.SA);
    double2* B = static_cast<double2*>(opm.SB);
    // 1. forward transform of the rows on the N grid into A: [c][rows_N][Hb]
    {
        FirstArgs<double> fa{};
        fa.done = nullptr;
        fa.g = gn;
        fa.ax = opn.ax[d - 1];
        const int rpb1 = opn.v2_row ? opn.rpb_first : opn.rpb;
        fa.rpb = rpb1;
        fa.npen = (rpb1 * d + 1) / 2;
        fa.x = xn;
        fa.A = opn.A;
        fa.out = reinterpret_cast<cpx<double>*>(A);
        fa.twg = static_cast<const cpx<double>*>(opn.tw[d - 1]);
        const unsigned nblk = (unsigned)((gn.rows + rpb1 - 1) / rpb1);
        if (d == 2)
            e = opn.v2_row ? v2_first<double, 2>(opn, fa, OP_ID, nblk) : launch_first<double, 2>(opn, fa, OP_ID, nblk);
        else
            e = opn.v2_row ? v2_first<double, 3>(opn, fa, OP_ID, nblk) : launch_first<double, 3>(opn, fa, OP_ID, nblk);
        if (e != hipSuccess) return e;
    }
    const int Hb = gn.Hb;  // (N_last + 1) / 2, the same band on both grids
    const int N0 = gn.L[0], M0 = gm.L[0];
    if (d == 3) {
        const int N1 = gn.L[1], M1 = gm.L[1];
        const long long colsN = (long long)N1 * Hb;
        // 2. forward along axis 1 (N1): A -> B
        if ((e = axis_custom(opn, opn.ax[1], opn.tw[1], false, N1, 0, N1, 0, Hb, N0, (long long)N1 * Hb,
                             (long long)N1 * Hb, gn.s1, gn.s1, A, B)) != hipSuccess)
            return e;
        // 3. forward along axis 0 (N0): B -> A, columns (k1, k2)
        if ((e = axis_custom(opn, opn.ax[0], opn.tw[0], false, N0, 0, N0, 0, (int)colsN, 1, 0, 0, N0 * colsN,
                             N0 * colsN, B, A)) != hipSuccess)
            return e;
        // 4. inverse along axis 0 on M0 from the N0 band: A -> B [c][M0][N1 Hb]
        if ((e = axis_custom(opm, opm.ax[0], opm.tw[0], true, N0, 1, M0, 0, (int)colsN, 1, 0, 0, N0 * colsN,
                             M0 * colsN, A, B)) != hipSuccess)
            return e;
        // 5. inverse along axis 1 on M1 from the N1 band: B -> A [c][M0][M1][Hb]
        if ((e = axis_custom(opm, opm.ax[1], opm.tw[1], true, N1, 1, M1, 0, Hb, M0, (long long)N1 * Hb,
                             (long long)M1 * Hb, M0 * colsN, gm.s1, B, A)) != hipSuccess)
            return e;
    } else {
        // 3. forward along axis 0 (N0): A -> B
        if ((e = axis_custom(opn, opn.ax[0], opn.tw[0], false, N0, 0, N0, 0, Hb, 1, 0, 0, (long long)N0 * Hb,
                             (long long)N0 * Hb, A, B)) != hipSuccess)
            return e;
        // 4. inverse along axis 0 on M0 from the band: B -> A [c][M0][Hb]
        if ((e = axis_custom(opm, opm.ax[0], opm.tw[0], true, N0, 1, M0, 0, Hb, 1, 0, 0, (long long)N0 * Hb,
                             (long long)M0 * Hb, B, A)) != hipSuccess)
            return e;
    }
    // 6. rows back to real values on the double grid, scaled by the forward factor 1/|N|
    LastArgs<double> la{};
    la.done = nullptr;
    la.sc = nullptr;
    la.g = gm;
    la.ax = opm.ax[d - 1];
    la.rpb = opm.rpb;
    la.npen = opm.npen;
    la.in = reinterpret_cast<const cpx<double>*>(A);
    la.y = ym;
    la.sgn = 1.0 / (double)gn.npts;
    la.A = opm.A;
    la.partials = opm.partials;
    la.twg = static_cast<const cpx<double>*>(opm.tw[d - 1]);
    unsigned nblk = (unsigned)((gm.rows + opm.rpb - 1) / opm.rpb);
    if (d == 2)
        return opm.v2_row ? v2_last<double, 2>(opm, la, EPI_STORE, &nblk) : launch_last<double, 2>(opm, la, EPI_STORE, nblk);
    return opm.v2_row ? v2_last<double, 3>(opm, la, EPI_STORE, &nblk) : launch_last<double, 3>(opm, la, EPI_STORE, nblk);
}

template <typename T>
hipError_t run_apply(const OpPlan& op, const ApplyArgs& a, int* nblocks_last)
{
    if (op.g.d == 2) return apply_d<T, 2>(op, a, nblocks_last);
    return apply_d<T, 3>(op, a, nblocks_last);
}
template hipError_t run_apply<float>(const OpPlan&, const ApplyArgs&, int*);
template hipError_t run_apply<double>(const OpPlan&, const ApplyArgs&, int*);

bool batchable(const OpPlan& op) { return op.v2_row && op.v2_mid && (op.g.d == 2 || op.v2_axis); }

template <typename T>
BatchTables<T> batch_tables(void* region)
{
    BatchTables<T> t{};
    char* base = static_cast<char*>(region);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base + off;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    t.fa = reinterpret_cast<FirstArgs<T>*>(take(kMaxBatch * sizeof(FirstArgs<T>)));
    t.xf = reinterpret_cast<AxisArgs<T>*>(take(kMaxBatch * sizeof(AxisArgs<T>)));
    t.xi = reinterpret_cast<AxisArgs<T>*>(take(kMaxBatch * sizeof(AxisArgs<T>)));
    t.ma = reinterpret_cast<MidArgs<T>*>(take(kMaxBatch * sizeof(MidArgs<T>)));
    t.la = reinterpret_cast<LastArgs<T>*>(take(kMaxBatch * sizeof(LastArgs<T>)));
    t.red = reinterpret_cast<ReduceArgs*>(take(kMaxBatch * sizeof(ReduceArgs)));
    t.red2 = reinterpret_cast<ReduceArgs*>(take(kMaxBatch * sizeof(ReduceArgs)));
    t.upd = reinterpret_cast<UpdateArgs<T>*>(take(kMaxBatch * sizeof(UpdateArgs<T>)));
    t.bytes = off;
    return t;
}
template BatchTables<float> batch_tables<float>(void*);
template BatchTables<double> batch_tables<double>(void*);
static_assert(kMaxBatch * (sizeof(FirstArgs<double>) + 2 * sizeof(AxisArgs<double>) + sizeof(MidArgs<double>) +
                           sizeof(LastArgs<double>) + 2 * sizeof(ReduceArgs) + sizeof(UpdateArgs<double>)) +
                      8 * 256 <=
                  kBatchSlabBytes,
              "batch tables exceed their region");

template <typename T>
hipError_t build_bundle(const OpPlan& op, const ApplyArgs& a, ApplyBundle<T>* out)
{
    if (op.g.d == 2) return build_bundle_d<T, 2>(op, a, out);
    return build_bundle_d<T, 3>(op, a, out);
}
template hipError_t build_bundle<float>(const OpPlan&, const ApplyArgs&, ApplyBundle<float>*);
template hipError_t build_bundle<double>(const OpPlan&, const ApplyArgs&, ApplyBundle<double>*);

template <typename T, int D>
static hipError_t apply_batch_d(const OpPlan& op, const ApplyBundle<T>& b0, const BatchTables<T>& t, int nb)
{
    const Geo& g = op.g;
    hipError_t e;
    if (!b0.skip_first && (e = v2_first_b<T, D>(op, t.fa, b0.op, b0.nblk1, nb)) != hipSuccess) return e;
    if (b0.first_only) return hipSuccess;
    if (D == 3 && (e = v2_axis_b<T>(op, t.xf, false, b0.xf.ntiles, g.L[0], g.B[1], nb)) != hipSuccess) return e;
    if ((e = v2_middle_b<T, D>(op, t.ma, b0.mult, b0.ma.ntiles, nb)) != hipSuccess) return e;
    if (D == 3 && (e = v2_axis_b<T>(op, t.xi, true, b0.xi.ntiles, g.L[0], g.B[1], nb)) != hipSuccess) return e;
    return v2_last_b<T, D>(op, t.la, b0.epi, b0.fused, b0.nblk_last, nb);
}

template <>
hipError_t run_apply_batch<float>(const OpPlan& op0, const ApplyBundle<float>& b0, const BatchTables<float>& t, int nb)
{
    if (!batchable(op0) || nb < 1 || nb > kMaxBatch) return hipErrorInvalidValue;
    if (op0.g.d == 2) return apply_batch_d<float, 2>(op0, b0, t, nb);
    return apply_batch_d<float, 3>(op0, b0, t, nb);
}

hipError_t run_reduce_batch(hipStream_t s, const ReduceArgs* tab, int nb, int redop)
{
    hipLaunchKernelGGL(k_reduce_b, dim3(nb), dim3(kThreads), 0, s, tab, redop);
    return hipGetLastError();
}

template <typename T>
hipError_t run_cg_update_batch(hipStream_t s, const UpdateArgs<T>* tab, int nb)
{
    hipLaunchKernelGGL(k_cg_update_b<T>, dim3(kVecBlocks, nb), dim3(kThreads), 0, s, tab);
    return hipGetLastError();
}
template hipError_t run_cg_update_batch<float>(hipStream_t, const UpdateArgs<float>*, int);


hipError_t run_init_loop(const OpPlan& op, double rr, double alpha, double beta, double thr, double npts,
                         double blowup, double cheb_c, double cheb_delta, int limit)
{
    hipLaunchKernelGGL(k_init_loop, dim3(1), dim3(1), 0, op.stream, op.sc, rr, alpha, beta, thr, npts, blowup, cheb_c,
                       cheb_delta, limit);
    return hipGetLastError();
}

hipError_t run_set_scalar(const OpPlan& op, double* dst, double v)
{
    hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, op.stream, dst, v);
    return hipGetLastError();
}

// A launch of a kernel that is not a pass, bracketed by the profiler's events while its kind is
// being timed (the events are attached to the dispatch itself, as for the passes).
#define LAUNCH_TIMED(KIND, OP, KERNEL, GRID, STREAM, ...)                                          \
    do {                                                                                        \
        const bool timed_ = (OP).prof && (OP).prof->wants(KIND);                                \
        if (timed_) {                                                                           \
            hipError_t e_ = (OP).prof->begin(KIND);                                             \
            if (e_ != hipSuccess) return e_;                                                    \
            const PassEvents pe_ = g_pass_events;                                               \
            g_pass_events = PassEvents{};                                                       \
            hipExtLaunchKernelGGL(KERNEL, GRID, dim3(kThreads), 0, (STREAM), pe_.start, pe_.stop, 0, __VA_ARGS__); \
            if ((e_ = hipGetLastError()) != hipSuccess) return e_;                              \
            if ((e_ = (OP).prof->end()) != hipSuccess) return e_;                               \
        } else {                                                                                \
            hipLaunchKernelGGL(KERNEL, GRID, dim3(kThreads), 0, (STREAM), __VA_ARGS__);          \
        }                                                                                       \
    } while (0)

hipError_t run_reduce_async(const OpPlan& op, int n, int redop)
{
    LAUNCH_TIMED(PK_REDUCE, op, k_reduce, dim3(1), op.stream, op.partials, n, op.sc, redop);
    return hipGetLastError();
}

hipError_t run_reduce(const OpPlan& op, int n, int redop, double* host_out)
{
    hipError_t e = run_reduce_async(op, n, redop);
    if (e != hipSuccess) return e;
    if (!host_out) return hipSuccess;
    e = hipMemcpyAsync(host_out, &op.sc->total, sizeof(double), hipMemcpyDeviceToHost, op.stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(op.stream);
}

template <typename T>
hipError_t run_cg_update(const OpPlan& op, long long n, T* x, T* r, const T* p, const T* q)
{
    LAUNCH_TIMED(PK_CG_UPDATE, op, k_cg_update<T>, dim3(kVecBlocks), op.stream, n, x, r, p, q, op.sc, op.partials);
    return hipGetLastError();
}
template hipError_t run_cg_update<float>(const OpPlan&, long long, float*, float*, const float*, const float*);
template hipError_t run_cg_update<double>(const OpPlan&, long long, double*, double*, const double*, const double*);

template <typename T>
hipError_t run_cg_x(const OpPlan& op, long long n, T* x, const T* p)
{
    hipLaunchKernelGGL(k_cg_x<T>, dim3(kVecBlocks), dim3(kThreads), 0, op.stream, n, x, p, op.sc);
    return hipGetLastError();
}
template hipError_t run_cg_x<float>(const OpPlan&, long long, float*, const float*);
template hipError_t run_cg_x<double>(const OpPlan&, long long, double*, const double*);

template <typename T>
hipError_t run_fill(hipStream_t s, long long n, T* x, T v)
{
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, v);
    return hipGetLastError();
}
template hipError_t run_fill<float>(hipStream_t, long long, float*, float);
template hipError_t run_fill<double>(hipStream_t, long long, double*, double);
template hipError_t run_fill<unsigned>(hipStream_t, long long, unsigned*, unsigned);

template <typename T>
hipError_t run_fill_field(hipStream_t s, int d, long long npts, T* x, const double* v)
{
    hipLaunchKernelGGL(k_fill_field<T>, dim3(grid_for(d * npts)), dim3(kThreads), 0, s, d, npts, x, v[0], v[1],
                       d == 3 ? v[2] : 0.0);
    return hipGetLastError();
}
template hipError_t run_fill_field<float>(hipStream_t, int, long long, float*, const double*);
template hipError_t run_fill_field<double>(hipStream_t, int, long long, double*, const double*);

template <typename T>
hipError_t run_copy(hipStream_t s, long long n, T* dst, const T* src)
{
    hipLaunchKernelGGL(k_copy<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, n, dst, src);
    return hipGetLastError();
}
template hipError_t run_copy<float>(hipStream_t, long long, float*, const float*);
template hipError_t run_copy<double>(hipStream_t, long long, double*, const double*);

hipError_t run_f64_to_f32(hipStream_t s, long long n, float* dst, const double* src)
{
    hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n)), dim3(kThreads), 0, s, n, dst, src);
    return hipGetLastError();
}

hipError_t run_twiddles(hipStream_t s, int L, double2* tw)
{
    hipLaunchKernelGGL(k_twiddles, dim3(grid_for(L)), dim3(kThreads), 0, s, L, tw);
    return hipGetLastError();
}

hipError_t run_add_f32_to_f64(hipStream_t s, long long n, double* x, const float* d)
{
    hipLaunchKernelGGL(k_add_f32_to_f64, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, d);
    return hipGetLastError();
}

hipError_t run_axpby(hipStream_t s, long long n, double* y, double a, const double* x, double b)
{
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kThreads), 0, s, n, y, a, x, b);
    return hipGetLastError();
}

hipError_t run_add_f64(hipStream_t s, long long n, double* x, const double* d)
{
    hipLaunchKernelGGL(k_add_f64, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, d);
    return hipGetLastError();
}

template <typename T>
hipError_t run_dot(const OpPlan& op, long long n, const T* a, const T* b, int* nblocks)
{
    hipLaunchKernelGGL(k_dot<T>, dim3(kVecBlocks), dim3(kThreads), 0, op.stream, n, a, b, op.partials);
    *nblocks = kVecBlocks;
    return hipGetLastError();
}
template hipError_t run_dot<float>(const OpPlan&, long long, const float*, const float*, int*);
template hipError_t run_dot<double>(const OpPlan&, long long, const double*, const double*, int*);

hipError_t run_norm_AE(const OpPlan& op, const double* E, int* nblocks)
{
    const long long n = op.g.npts;
    const int d = op.g.d;
    const int k = op.A.kind;
#define NAE(DD, KK) hipLaunchKernelGGL((k_norm_AE<DD, KK>), dim3(kVecBlocks), dim3(kThreads), 0, op.stream, n, op.A, E[0], E[1], d == 3 ? E[2] : 0.0, op.partials)
    if (d == 2) {
        if (k == AK_SYM) NAE(2, AK_SYM); else if (k == AK_ISO) NAE(2, AK_ISO); else NAE(2, AK_PHASE);
    } else {
        if (k == AK_SYM) NAE(3, AK_SYM); else if (k == AK_ISO) NAE(3, AK_ISO); else NAE(3, AK_PHASE);
    }
#undef NAE
    *nblocks = kVecBlocks;
    return hipGetLastError();
}

hipError_t run_effective(const OpPlan& op, int nrhs, const double* E, const double* e, int* nblocks)
{
    const long long n = op.g.npts;
    const int d = op.g.d;
    const int k = op.A.kind;
    const int nb = 512;
#define EFF(DD, KK) hipLaunchKernelGGL((k_effective<DD, KK>), dim3(nb), dim3(kThreads), 0, op.stream, n, op.A, nrhs, E, e, op.partials)
    if (d == 2) {
        if (k == AK_SYM) EFF(2, AK_SYM); else if (k == AK_ISO) EFF(2, AK_ISO); else EFF(2, AK_PHASE);
    } else {
        if (k == AK_SYM) EFF(3, AK_SYM); else if (k == AK_ISO) EFF(3, AK_ISO); else EFF(3, AK_PHASE);
    }
#undef EFF
    *nblocks = nb;
    return hipGetLastError();
}

// Non-conformity of an iterate (Sec. 4.4): partials [block][1 + D] of |y - (x - s)|^2 with
// y = G x, and of the components of x (for its mean); s = E when x is the whole Eyre-Milton field
// (G removes the mean, so G x = G (x - E)), s = 0 for a fluctuation.
template <int D>
__global__ __launch_bounds__(kThreads) void k_nonconf(long long npts, const double* __restrict__ y,
                                                      const double* __restrict__ x, const double* shift,
                                                      double* partials)
{
    __shared__ double red[kThreads / 64];
    double sh[D];
#pragma unroll
    for (int c = 0; c < D; c++) sh[c] = shift[c];
    double acc[1 + D];
#pragma unroll
    for (int q = 0; q <= D; q++) acc[q] = 0.0;
    for (long long pt = (long long)blockIdx.x * blockDim.x + threadIdx.x; pt < npts; pt += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < D; c++) {
            const double xv = x[c * npts + pt];
            const double dv = y[c * npts + pt] - (xv - sh[c]);
            acc[0] += dv * dv;
            acc[1 + c] += xv;
        }
    }
#pragma unroll
    for (int q = 0; q <= D; q++) {
        const double tot = block_sum(acc[q], red);
        if (threadIdx.x == 0) partials[(long long)blockIdx.x * (1 + D) + q] = tot;
        __syncthreads();
    }
}

// History entries of the non-conformity: nc = ||G x - (x - s)||_2 and mean = |<x> - s| (the
// mean-value component of the Helmholtz split of the Eyre-Milton error), at slot base + m mod cap.
template <int D>
__global__ __launch_bounds__(kThreads) void k_hist_nc(const double* __restrict__ partials, int nb, const Scalars* s,
                                                      const double* shift, double* nc, double* mean, int cap,
                                                      double inv_npts)
{
    __shared__ double red[kThreads / 64];
    double tot[1 + D];
#pragma unroll
    for (int q = 0; q <= D; q++) {
        double v = 0.0;
        for (int i = threadIdx.x; i < nb; i += blockDim.x) v += partials[(long long)i * (1 + D) + q];
        tot[q] = block_sum(v, red);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const long long slot = (long long)s->aux[14] + s->m % cap;
        if (nc) nc[slot] = sqrt(tot[0] * inv_npts);
        if (mean) {
            double m2 = 0.0;
#pragma unroll
            for (int c = 0; c < D; c++) {
                const double dm = tot[1 + c] * inv_npts - shift[c];
                m2 += dm * dm;
            }
            mean[slot] = sqrt(m2);
        }
    }
}

hipError_t run_hist_nonconf(const OpPlan& op, const double* x, const double* shift, double* y, double* nc,
                            double* mean, int cap)
{
    // y = G x (y: a vector of the integration grid)
    ApplyArgs a;
    a.op = OP_ID;
    a.x = x;
    a.mult = MULT_G;
    a.epi = EPI_STORE;
    a.sgn = 1.0;
    a.y = y;
    int nb = 0;
    hipError_t e = run_apply<double>(op, a, &nb);
    if (e != hipSuccess) return e;
    const int nbk = 512;
    if (op.g.d == 2) {
        hipLaunchKernelGGL(k_nonconf<2>, dim3(nbk), dim3(kThreads), 0, op.stream, op.g.npts, y, x, shift, op.partials);
        hipLaunchKernelGGL(k_hist_nc<2>, dim3(1), dim3(kThreads), 0, op.stream, op.partials, nbk, op.sc, shift, nc, mean,
                           cap, 1.0 / (double)op.g.npts);
    } else {
        hipLaunchKernelGGL(k_nonconf<3>, dim3(nbk), dim3(kThreads), 0, op.stream, op.g.npts, y, x, shift, op.partials);
        hipLaunchKernelGGL(k_hist_nc<3>, dim3(1), dim3(kThreads), 0, op.stream, op.partials, nbk, op.sc, shift, nc, mean,
                           cap, 1.0 / (double)op.g.npts);
    }
    return hipGetLastError();
}

// One entry of a solver's history at body count m = s->m, slot base + m mod cap: the stopping-test
// quantity (s->last times aux[12]; aux[13] before the first body) and, when `en` is set, the
// energy reduced from the first of the nvals interleaved partial sums, times en_scale.
__global__ __launch_bounds__(kThreads) void k_hist(const double* __restrict__ partials, int nb, int nvals,
                                                   const Scalars* s, double* res, double* en, int cap,
                                                   double en_scale)
{
    __shared__ double red[kThreads / 64];
    double v = 0.0;
    if (en)
        for (int i = threadIdx.x; i < nb; i += blockDim.x) v += partials[(long long)i * nvals];
    const double tot = block_sum(v, red);
    if (threadIdx.x == 0) {
        const int m = s->m;
        const long long slot = (long long)s->aux[14] + m % cap;
        if (res) res[slot] = m == 0 ? s->aux[13] : s->last * s->aux[12];
        if (en) en[slot] = tot * en_scale;
    }
}

hipError_t run_hist(hipStream_t stream, const double* partials, int nb, int nvals, const Scalars* sc, double* res,
                    double* en, int cap, double en_scale)
{
    hipLaunchKernelGGL(k_hist, dim3(1), dim3(kThreads), 0, stream, partials, nb, nvals, sc, res, en, cap, en_scale);
    return hipGetLastError();
}

hipError_t run_reduce_multi(const OpPlan& op, int nblocks, int nvals, double* host_out)
{
    double* dev_out = op.sc->aux + 16;
    hipLaunchKernelGGL(k_reduce_multi, dim3(1), dim3(kThreads), 0, op.stream, op.partials, nblocks, nvals, dev_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(host_out, dev_out, sizeof(double) * nvals, hipMemcpyDeviceToHost, op.stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(op.stream);
}

hipError_t run_to_f32(hipStream_t s, long long n, float* dst, const double* src)
{
    hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(kThreads), 0, s, n, dst, src);
    return hipGetLastError();
}

hipError_t run_eig_bounds(hipStream_t s, int d, int kind, const double* coef, long long npts, double* partials,
                          int* nblocks)
{
    const unsigned nb = grid_for(npts, kThreads, 1024);
    if (d == 2)
        hipLaunchKernelGGL(k_eig_bounds<2>, dim3(nb), dim3(kThreads), 0, s, kind, coef, npts, partials);
    else
        hipLaunchKernelGGL(k_eig_bounds<3>, dim3(nb), dim3(kThreads), 0, s, kind, coef, npts, partials);
    *nblocks = (int)nb;
    return hipGetLastError();
}

hipError_t run_minmax_reduce(hipStream_t s, const double* partials, int nblocks, double* host_lo_hi)
{
    double* dev = const_cast<double*>(partials) + 2 * nblocks;
    hipLaunchKernelGGL(k_minmax, dim3(1), dim3(kThreads), 0, s, partials, nblocks, dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(host_lo_hi, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

hipError_t run_phase_mask(hipStream_t s, const uint8_t* phase, long long npts, unsigned* mask)
{
    hipLaunchKernelGGL(k_phase_mask, dim3(grid_for(npts, kThreads, 1024)), dim3(kThreads), 0, s, phase, npts, mask);
    return hipGetLastError();
}

hipError_t run_ga_component(hipStream_t s, const GaAsm& ga, int kind, const double* coef, int comp,
                            const uint8_t* phase, const double* pv, int nphase, double* out)
{
    double v[16] = {0};
    for (int i = 0; i < nphase && i < 16; i++) v[i] = pv[i];
    hipLaunchKernelGGL(k_coef_component, dim3(grid_for(ga.nN)), dim3(kThreads), 0, s, ga.nN, kind, coef, comp, phase,
                       v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9], v[10], v[11], v[12], v[13], v[14],
                       v[15], ga.c0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // forward DFT on the N grid (with 1/|N|), axis by axis, ping-pong c0 <-> c1
    double2* src = ga.c0;
    double2* dst = ga.c1;
    for (int a = 0; a < ga.d; a++) {
        long long stride = 1;
        for (int b = a + 1; b < ga.d; b++) stride *= ga.N[b];
        const double scale = (a == 0) ? 1.0 / (double)ga.nN : 1.0;
        hipLaunchKernelGGL(k_dft_axis, dim3(grid_for(ga.nN)), dim3(kThreads), 0, s, src, dst, ga.nN, ga.N[a], stride,
                           ga.twN[a], -1, scale);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        double2* t = src;
        src = dst;
        dst = t;
    }
    // periodic extension with sinc weights onto the double-grid frequencies
    hipLaunchKernelGGL(k_ga_extend, dim3(grid_for(ga.nM)), dim3(kThreads), 0, s, src, dst, ga.d, ga.N[0], ga.N[1],
                       ga.d == 3 ? ga.N[2] : 1, ga.M[0], ga.M[1], ga.d == 3 ? ga.M[2] : 1, ga.sinc[0], ga.sinc[1],
                       ga.d == 3 ? ga.sinc[2] : ga.sinc[1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {
        double2* t = src;
        src = dst;
        dst = t;
    }
    for (int a = 0; a < ga.d; a++) {
        long long stride = 1;
        for (int b = a + 1; b < ga.d; b++) stride *= ga.M[b];
        hipLaunchKernelGGL(k_dft_axis, dim3(grid_for(ga.nM)), dim3(kThreads), 0, s, src, dst, ga.nM, ga.M[a], stride,
                           ga.twM[a], +1, 1.0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        double2* t = src;
        src = dst;
        dst = t;
    }
    hipLaunchKernelGGL(k_real_part, dim3(grid_for(ga.nM)), dim3(kThreads), 0, s, ga.nM, src, out);
    return hipGetLastError();
}

}  // namespace fgh
