// fgh_fft.hpp -- LDS-resident mixed-radix Stockham FFT for odd lengths (gfx950, wave64).
//
// A workgroup transforms P pencils of length L held in LDS (pencil p at offset p * L).
// Each stage of radix R (product of the earlier radices Ns) reads butterfly inputs j + r L/R,
// multiplies by the twiddles exp(-+2 pi i (j mod Ns) r / (Ns R)), applies the radix-R DFT and
// writes outputs at (j - j mod Ns) R + j mod Ns + r Ns into the other LDS buffer (Stockham
// auto-sort: no bit reversal, natural order in and out).  Radices 3, 5, 7 use closed-form
// butterflies with compile-time roots; any other odd prime uses a direct sum whose roots come
// from the twiddle table.  All lengths on the hot path (63, 125, 135, 243, 45, 81, 729) factor
// into 3, 5 and 7.
#pragma once
#include <hip/hip_runtime.h>

#include "fgh_internal.hpp"

namespace fgh {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }
// -i * a
template <typename T>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) { return {a.y, -a.x}; }

// cos(2 pi m / R) and sin(2 pi m / R) for R in {3, 5, 7}, 0 < m < R.
__device__ __forceinline__ constexpr double root_cos(int R, int m)
{
    if (R == 3) return -0.5;
    if (R == 5) return (m == 1 || m == 4) ? 0.30901699437494742410229341718281906
                                          : -0.80901699437494742410229341718281906;
    // R == 7
    return (m == 1 || m == 6) ? 0.62348980185873353052500488400423981
         : (m == 2 || m == 5) ? -0.22252093395631440428890256449679476
                              : -0.90096886790241912623610231950744505;
}
__device__ __forceinline__ constexpr double root_sin(int R, int m)
{
    if (R == 3) return m == 1 ? 0.86602540378443864676372317075293618 : -0.86602540378443864676372317075293618;
    if (R == 5) {
        const double s1 = 0.95105651629515357211643933337938214, s2 = 0.58778525229247312916870595463907277;
        return m == 1 ? s1 : m == 2 ? s2 : m == 3 ? -s2 : -s1;
    }
    const double s1 = 0.78183148246802980870844452667405775, s2 = 0.97492791218182360701813168299393122,
                 s3 = 0.43388373911755812047576833284835875;
    return m == 1 ? s1 : m == 2 ? s2 : m == 3 ? s3 : m == 4 ? -s3 : m == 5 ? -s2 : -s1;
}

// In-register radix-R DFT (R odd), forward sign exp(-2 pi i jk/R) unless INV.
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_small(cpx<T>* v)
{
    constexpr int H = (R - 1) / 2;
    cpx<T> a[H], b[H];
#pragma unroll
    for (int k = 1; k <= H; k++) {
        a[k - 1] = v[k] + v[R - k];
        b[k - 1] = v[k] - v[R - k];
    }
    cpx<T> out[R];
    cpx<T> y0 = v[0];
#pragma unroll
    for (int k = 1; k <= H; k++) y0 = y0 + a[k - 1];
    out[0] = y0;
#pragma unroll
    for (int j = 1; j <= H; j++) {
        cpx<T> re = v[0];
        cpx<T> im = {T(0), T(0)};
#pragma unroll
        for (int k = 1; k <= H; k++) {
            const int m = (j * k) % R;
            re = re + T(root_cos(R, m)) * a[k - 1];
            im = im + T(root_sin(R, m)) * b[k - 1];
        }
        const cpx<T> mi = mul_mi(im);
        if (!INV) {
            out[j] = re + mi;
            out[R - j] = re - mi;
        } else {
            out[j] = re - mi;
            out[R - j] = re + mi;
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++) v[r] = out[r];
}

template <typename T, bool INV>
__device__ __forceinline__ cpx<T> twiddle(const cpx<T>* tw, int m)
{
    cpx<T> w = tw[m];
    return INV ? conj(w) : w;
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void stage_small(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                            int L, int Ns, int P, const cpx<T>* tw)
{
    const int nb = L / R;
    const int tot = nb * P;
    const int tstep = L / (Ns * R);
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        const int p = t / nb;
        const int j = t - p * nb;
        const int k = (Ns == 1) ? 0 : j % Ns;
        const cpx<T>* s = src + p * L;
        cpx<T>* o = dst + p * L;
        cpx<T> v[R];
        v[0] = s[j];
#pragma unroll
        for (int r = 1; r < R; r++) {
            v[r] = s[j + r * nb];
            if (k) v[r] = cmul(v[r], twiddle<T, INV>(tw, r * k * tstep));
        }
        dft_small<T, R, INV>(v);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; r++) o[base + r * Ns] = v[r];
    }
}

// Any odd radix R dividing L (used for primes > 7): direct sum, roots from the table.
template <typename T, bool INV>
__device__ void stage_generic(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst, int R, int L,
                              int Ns, int P, const cpx<T>* tw)
{
    const int nb = L / R;
    const int tot = nb * P;
    const int tstep = L / (Ns * R);
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        const int p = t / nb;
        const int j = t - p * nb;
        const int k = j % Ns;
        const cpx<T>* s = src + p * L;
        cpx<T>* o = dst + p * L;
        const int base = (j - k) * R + k;
        for (int q = 0; q < R; q++) {
            cpx<T> acc = {T(0), T(0)};
            for (int r = 0; r < R; r++) {
                cpx<T> v = s[j + r * nb];
                if (k && r) v = cmul(v, twiddle<T, INV>(tw, r * k * tstep));
                acc = acc + cmul(v, twiddle<T, INV>(tw, ((r * q) % R) * nb));
            }
            o[base + q * Ns] = acc;
        }
    }
}

// Transform P pencils of length ax.L starting in buffer a (b is scratch of the same size).
// Returns the buffer holding the result (a if the number of stages is even, else b).
// Callers synchronise before the call; the call ends with a barrier.
template <typename T, bool INV>
__device__ cpx<T>* fft_lds(cpx<T>* a, cpx<T>* b, const Axis& ax, int P, const cpx<T>* tw)
{
    cpx<T>* src = a;
    cpx<T>* dst = b;
    int Ns = 1;
    const int L = ax.L;
    for (int s = 0; s < ax.nst; s++) {
        const int R = ax.rad[s];
        if (R == 3)
            stage_small<T, 3, INV>(src, dst, L, Ns, P, tw);
        else if (R == 5)
            stage_small<T, 5, INV>(src, dst, L, Ns, P, tw);
        else if (R == 7)
            stage_small<T, 7, INV>(src, dst, L, Ns, P, tw);
        else
            stage_generic<T, INV>(src, dst, R, L, Ns, P, tw);
        __syncthreads();
        cpx<T>* t = src;
        src = dst;
        dst = t;
        Ns *= R;
    }
    return src;
}

// Deterministic block sum (fixed shuffle tree, then waves in order).  Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; i++) tot += red[i];
    }
    return tot;
}

__device__ __forceinline__ int signed_index(int i, int n) { return (2 * i < n) ? i : i - n; }

// Stored band index s in [0, B) -> position in an FFT of length L (frequency signed(s, B)).
__device__ __forceinline__ int band_pos(int s, int B, int L)
{
    const int k = signed_index(s, B);
    return k < 0 ? k + L : k;
}

}  // namespace fgh
