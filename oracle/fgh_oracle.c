/*
 * fgh_oracle.c -- plain, slow FP64 CPU oracle for Fourier-Galerkin FFT homogenization
 * (Mishra, Vondrejc, Zeman, "A comparative study on low-memory iterative solvers for
 * FFT-based homogenization of periodic media", arXiv 1508.02045).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library.  It shares no code with the GPU path: it has its
 * own naive discrete Fourier transform (direct sums), its own projection, coefficient
 * assembly, solvers and reductions.  Everything is double precision, full complex arrays,
 * no blocking and no fusion, so that each step can be checked against the paper by eye.
 *
 * Conventions (paper Sec. 2.1):
 *   - d in {2,3}; every N_a odd.  A grid of n_a points per axis; point index i_a in [0,n_a)
 *     stands for the signed index m_a = i_a if 2 i_a < n_a else i_a - n_a, and the grid point
 *     x_a = m_a / n_a (paper: grid points x_N^m = m/N, cell (-1/2,1/2)^d).
 *   - Arrays are C-order over the grid; a vector field is [d][grid], a coefficient field is
 *     [grid][d][d] (row-major d x d block per point).
 *   - Forward DFT carries 1/|grid| and exp(-2 pi i m k / n); the inverse has exp(+...) and no
 *     factor (eq:DFT).  Frequency index i <-> integer frequency k = signed(i).
 *   - Inner product (a,b)_2 = (1/|grid|) sum_points a.b (Notation paragraph); the grid is N
 *     for GaNi and the double grid M = 2N-1 for Ga.
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_GANI 0
#define ORC_GA 1

#define ORC_RICHARDSON 0
#define ORC_CG 1
#define ORC_CHEBYSHEV 2
#define ORC_EYRE_MILTON 3

#define ORC_OK 0
#define ORC_E_INVALID 1
#define ORC_E_NO_CONVERGENCE 5
#define ORC_E_DIVERGED 6

typedef double complex cplx;

typedef struct {
    int d;
    int n[3];
    long size;
} grid_t;

static int mk_grid(int d, const int* n, grid_t* g)
{
    if (d < 1 || d > 3) return ORC_E_INVALID;
    g->d = d;
    g->size = 1;
    for (int a = 0; a < 3; a++) g->n[a] = 1;
    for (int a = 0; a < d; a++) {
        if (n[a] < 1 || n[a] % 2 == 0) return ORC_E_INVALID;
        g->n[a] = n[a];
        g->size *= n[a];
    }
    return ORC_OK;
}

/* Double grid M = 2N - 1 (eq:Ga_exact_integration). */
static int mk_double_grid(int d, const int* N, grid_t* g)
{
    int m[3];
    for (int a = 0; a < d; a++) m[a] = 2 * N[a] - 1;
    return mk_grid(d, m, g);
}

/* Signed frequency / index of position i on an odd axis of length n (eq:grid). */
static int signed_index(int i, int n) { return (2 * i < n) ? i : i - n; }

/* Multi-index of a flat C-order position. */
static void unflatten(const grid_t* g, long p, int* idx)
{
    for (int a = g->d - 1; a >= 0; a--) {
        idx[a] = (int)(p % g->n[a]);
        p /= g->n[a];
    }
}

/* ---------------------------------------------------------------------------------------- */
/* Naive DFT (eq:DFT): direct sums along one axis at a time.                                 */
/* ---------------------------------------------------------------------------------------- */

/* Along axis `ax`: X[k] = sum_j x[j] exp(sign 2 pi i j k / n), no scaling.  The root of unity
 * for (j k mod n) is evaluated in long double so that the table is correctly rounded. */
static void dft_axis(const grid_t* g, int ax, cplx* c, int sign)
{
    const int n = g->n[ax];
    long stride = 1;
    for (int a = ax + 1; a < g->d; a++) stride *= g->n[a];
    const long nlines = g->size / n;
    cplx* tw = (cplx*)malloc(sizeof(cplx) * n);
    for (int m = 0; m < n; m++) {
        long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)n;
        tw[m] = (double)cosl(ang) + (double)(sign * sinl(ang)) * I;
    }
#pragma omp parallel
    {
        cplx* tmp = (cplx*)malloc(sizeof(cplx) * n);
#pragma omp for schedule(static)
        for (long line = 0; line < nlines; line++) {
            long outer = line / stride, inner = line % stride;
            long base = outer * (long)n * stride + inner;
            for (int k = 0; k < n; k++) {
                cplx acc = 0.0;
                for (int j = 0; j < n; j++) acc += c[base + (long)j * stride] * tw[((long)j * k) % n];
                tmp[k] = acc;
            }
            for (int k = 0; k < n; k++) c[base + (long)k * stride] = tmp[k];
        }
        free(tmp);
    }
    free(tw);
}

/* F (forward, with 1/|grid|) or F^{-1} (inverse, no factor) over every axis. */
static void dft_nd(const grid_t* g, cplx* c, int inverse)
{
    for (int a = 0; a < g->d; a++) dft_axis(g, a, c, inverse ? +1 : -1);
    if (!inverse) {
        const double s = 1.0 / (double)g->size;
        for (long p = 0; p < g->size; p++) c[p] *= s;
    }
}

/* Exported for the tests: in-place DFT of a complex grid given as separate re/im arrays. */
int orc_dft(int d, const int* n, double* re, double* im, int inverse)
{
    grid_t g;
    if (mk_grid(d, n, &g)) return ORC_E_INVALID;
    cplx* c = (cplx*)malloc(sizeof(cplx) * g.size);
    for (long p = 0; p < g.size; p++) c[p] = re[p] + im[p] * I;
    dft_nd(&g, c, inverse);
    for (long p = 0; p < g.size; p++) {
        re[p] = creal(c[p]);
        im[p] = cimag(c[p]);
    }
    free(c);
    return ORC_OK;
}

/* Selected Fourier coefficients of the GaNi operator, by direct sums (eq:DFT, eq:linsys):
 * for each listed frequency k (signed integers, |k_a| <= (N_a - 1)/2),
 *   w(k) = G(k) zhat(k),  zhat(k) = (1/|N|) sum_m (A x)(m) exp(-2 pi i k.m / N),
 * with G(k) = k k^T / (k.k) and G(0) = 0.  A: [grid][d][d]; x: [d][grid]; ks: [nk][d];
 * out: [nk][d][2] (real, imaginary).  Full-size applies are checked at sampled frequencies
 * with it: one coefficient costs one pass over the grid and no transform. */
int orc_apply_at(int d, const int* N, const double* A, const double* x, int nk, const int* ks, double* out)
{
    grid_t g;
    if (mk_grid(d, N, &g) || nk < 1) return ORC_E_INVALID;
    const long S = g.size;
    for (int q = 0; q < nk; q++)
        for (int a = 0; a < d; a++)
            if (2 * abs(ks[q * d + a]) >= N[a]) return ORC_E_INVALID;
    /* per axis and frequency: exp(-2 pi i k m / n) for m in [0, n) */
    cplx* w = (cplx*)malloc(sizeof(cplx) * (size_t)nk * 3 * 8192);
    for (int q = 0; q < nk; q++)
        for (int a = 0; a < d; a++)
            for (int m = 0; m < N[a]; m++) {
                /* the root from the exact residue (k m mod n), in long double, then rounded */
                long km = ((long)ks[q * d + a] * m) % N[a];
                if (km < 0) km += N[a];
                const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)km / (long double)N[a];
                w[((size_t)q * 3 + a) * 8192 + m] = (double)cosl(ang) - (double)sinl(ang) * I;
            }
    cplx* acc = (cplx*)calloc((size_t)nk * d, sizeof(cplx));
#pragma omp parallel
    {
        cplx* loc = (cplx*)calloc((size_t)nk * d, sizeof(cplx));
#pragma omp for schedule(static)
        for (long p = 0; p < S; p++) {
            int idx[3] = {0, 0, 0};
            unflatten(&g, p, idx);
            double z[3];
            for (int a = 0; a < d; a++) {
                double v = 0.0;
                for (int b = 0; b < d; b++) v += A[(p * d + a) * d + b] * x[b * S + p];
                z[a] = v;
            }
            for (int q = 0; q < nk; q++) {
                cplx e = 1.0;
                for (int a = 0; a < d; a++) e *= w[((size_t)q * 3 + a) * 8192 + idx[a]];
                for (int a = 0; a < d; a++) loc[q * d + a] += z[a] * e;
            }
        }
#pragma omp critical
        for (int q = 0; q < nk * d; q++) acc[q] += loc[q];
        free(loc);
    }
    for (int q = 0; q < nk; q++) {
        const int* k = ks + q * d;
        double kk = 0.0;
        for (int a = 0; a < d; a++) kk += (double)k[a] * k[a];
        cplx kz = 0.0;
        for (int a = 0; a < d; a++) kz += (double)k[a] * acc[q * d + a] / (double)S;
        for (int a = 0; a < d; a++) {
            const cplx v = kk > 0.0 ? (double)k[a] * kz / kk : 0.0;
            out[(q * d + a) * 2] = creal(v);
            out[(q * d + a) * 2 + 1] = cimag(v);
        }
    }
    free(acc);
    free(w);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------- */
/* Projection (eq:proj, eq:discrete_proj).                                                    */
/* ---------------------------------------------------------------------------------------- */

/* In Fourier space on grid g, for each frequency k (signed index per axis):
 *   mode 0: w = G(k) z,        G(0) = 0, G(k) = k k^T / (k.k)
 *   mode 1: w = (I - 2 G(k)) z (the reflection of Alg. 4; the k = 0 mode passes unchanged)
 * For Ga (band != NULL) the multiplier is zero for frequencies outside Z_N, i.e. where some
 * |k_a| > (N_a - 1)/2 (eq:discrete_proj). */
static void fourier_multiplier(const grid_t* g, const int* band, cplx* const* zh, int mode)
{
    const int d = g->d;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < g->size; p++) {
        int idx[3], k[3] = {0, 0, 0};
        unflatten(g, p, idx);
        int outside = 0;
        double kk = 0.0;
        for (int a = 0; a < d; a++) {
            k[a] = signed_index(idx[a], g->n[a]);
            if (band && 2 * abs(k[a]) > band[a] - 1) outside = 1;
            kk += (double)k[a] * (double)k[a];
        }
        cplx z[3], w[3];
        for (int a = 0; a < d; a++) z[a] = zh[a][p];
        if (outside) {
            for (int a = 0; a < d; a++) w[a] = 0.0;
        } else if (kk == 0.0) {
            for (int a = 0; a < d; a++) w[a] = (mode == 0) ? 0.0 : z[a];
        } else {
            cplx kz = 0.0;
            for (int a = 0; a < d; a++) kz += (double)k[a] * z[a];
            for (int a = 0; a < d; a++) {
                cplx gz = (double)k[a] * kz / kk;
                w[a] = (mode == 0) ? gz : z[a] - 2.0 * gz;
            }
        }
        for (int a = 0; a < d; a++) zh[a][p] = w[a];
    }
}

/* y = Re F^{-1} [ multiplier . F z ] for a real vector field z [d][grid]. */
static void spectral_op(const grid_t* g, const int* band, const double* z, double* y, int mode)
{
    const int d = g->d;
    cplx* buf[3];
    for (int a = 0; a < d; a++) {
        buf[a] = (cplx*)malloc(sizeof(cplx) * g->size);
        for (long p = 0; p < g->size; p++) buf[a][p] = z[a * g->size + p];
        dft_nd(g, buf[a], 0);
    }
    fourier_multiplier(g, band, buf, mode);
    for (int a = 0; a < d; a++) {
        dft_nd(g, buf[a], 1);
        for (long p = 0; p < g->size; p++) y[a * g->size + p] = creal(buf[a][p]);
        free(buf[a]);
    }
}

/* Pointwise z(x) = A(x) v(x) with A given as [grid][d][d]. */
static void pointwise_A(const grid_t* g, const double* A, const double* v, double* z)
{
    const int d = g->d;
    const long S = g->size;
    for (long p = 0; p < S; p++)
        for (int a = 0; a < d; a++) {
            double s = 0.0;
            for (int b = 0; b < d; b++) s += A[(p * d + a) * d + b] * v[b * S + p];
            z[a * S + p] = s;
        }
}

static int op_grid(int d, const int* N, int rule, grid_t* g)
{
    if (rule == ORC_GANI) return mk_grid(d, N, g);
    if (rule == ORC_GA) {
        grid_t gn;
        if (mk_grid(d, N, &gn)) return ORC_E_INVALID;
        return mk_double_grid(d, N, g);
    }
    return ORC_E_INVALID;
}

/* The system operator C x = G A x (eq:linsys): GaNi on the N grid, Ga on the 2N-1 grid with
 * the band-limited projection G_{N,2N-1}.  A is the coefficient on that grid. */
int orc_apply(int d, const int* N, int rule, const double* A, const double* x, double* y)
{
    grid_t g;
    if (op_grid(d, N, rule, &g)) return ORC_E_INVALID;
    double* z = (double*)malloc(sizeof(double) * d * g.size);
    pointwise_A(&g, A, x, z);
    spectral_op(&g, rule == ORC_GA ? N : NULL, z, y, 0);
    free(z);
    return ORC_OK;
}

/* The projection alone, y = G x (used to check G^2 = G, self-adjointness, conformity). */
int orc_project(int d, const int* N, int rule, const double* x, double* y)
{
    grid_t g;
    if (op_grid(d, N, rule, &g)) return ORC_E_INVALID;
    spectral_op(&g, rule == ORC_GA ? N : NULL, x, y, 0);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------- */
/* Coefficients.                                                                              */
/* ---------------------------------------------------------------------------------------- */

/* Ga coefficients on the double grid (eq:Ga_exact_integration) for a pixel-wise constant A:
 * the exact Fourier coefficient of a function constant on each pixel of width 1/N_a centred at
 * m/N_a is  A^(n) = [prod_a sinc(n_a / N_a)] (1/|N|) sum_m A_m exp(-2 pi i n.m/N),
 * sinc t = sin(pi t)/(pi t); then A_M(y_j) = sum_{n in Z_M} A^(n) exp(2 pi i n.j/M) on the
 * double grid.  Done entry by entry of the d x d block.  Input [N grid][d][d], output
 * [M grid][d][d]. */
int orc_ga_assemble(int d, const int* N, const double* A_N, double* A_M)
{
    grid_t gn, gm;
    if (mk_grid(d, N, &gn) || mk_double_grid(d, N, &gm)) return ORC_E_INVALID;
    cplx* an = (cplx*)malloc(sizeof(cplx) * gn.size);
    cplx* am = (cplx*)malloc(sizeof(cplx) * gm.size);
    const long double PI = 3.141592653589793238462643383279502884L;
    for (int r = 0; r < d; r++)
        for (int c = 0; c < d; c++) {
            for (long p = 0; p < gn.size; p++) an[p] = A_N[(p * d + r) * d + c];
            dft_nd(&gn, an, 0);
            for (long q = 0; q < gm.size; q++) {
                int idx[3], src[3];
                unflatten(&gm, q, idx);
                double w = 1.0;
                for (int a = 0; a < d; a++) {
                    int nf = signed_index(idx[a], gm.n[a]); /* |nf| <= N_a - 1 */
                    if (nf != 0) {
                        long double t = PI * (long double)nf / (long double)N[a];
                        w *= (double)(sinl(t) / t);
                    }
                    src[a] = ((nf % N[a]) + N[a]) % N[a];
                }
                long sp = 0;
                for (int a = 0; a < d; a++) sp = sp * gn.n[a] + src[a];
                am[q] = w * an[sp];
            }
            dft_nd(&gm, am, 1);
            for (long q = 0; q < gm.size; q++) A_M[(q * d + r) * d + c] = creal(am[q]);
        }
    free(an);
    free(am);
    return ORC_OK;
}

/* Prolongation R_{N,M} = I_M o I_N^{-1} (eq:ev_bounds_GaNi): trigonometric interpolation of a
 * field given at the N grid, evaluated at the double grid.  u_N [d][N grid] -> u_M [d][M grid]. */
int orc_prolong(int d, const int* N, const double* uN, double* uM)
{
    grid_t gn, gm;
    if (mk_grid(d, N, &gn) || mk_double_grid(d, N, &gm)) return ORC_E_INVALID;
    cplx* cn = (cplx*)malloc(sizeof(cplx) * gn.size);
    cplx* cm = (cplx*)malloc(sizeof(cplx) * gm.size);
    for (int a = 0; a < d; a++) {
        for (long p = 0; p < gn.size; p++) cn[p] = uN[a * gn.size + p];
        dft_nd(&gn, cn, 0);
        for (long q = 0; q < gm.size; q++) cm[q] = 0.0;
        for (long p = 0; p < gn.size; p++) {
            int idx[3];
            unflatten(&gn, p, idx);
            long q = 0;
            for (int b = 0; b < d; b++) {
                int k = signed_index(idx[b], gn.n[b]);
                q = q * gm.n[b] + ((k % gm.n[b]) + gm.n[b]) % gm.n[b];
            }
            cm[q] = cn[p];
        }
        dft_nd(&gm, cm, 1);
        for (long q = 0; q < gm.size; q++) uM[a * gm.size + q] = creal(cm[q]);
    }
    free(cn);
    free(cm);
    return ORC_OK;
}

/* Eigenvalues of a symmetric d x d matrix by cyclic Jacobi rotations (textbook). */
static void sym_eig(int d, const double* Ain, double* ev)
{
    double a[3][3];
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) a[i][j] = 0.5 * (Ain[i * d + j] + Ain[j * d + i]);
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0.0;
        for (int i = 0; i < d; i++)
            for (int j = i + 1; j < d; j++) off += a[i][j] * a[i][j];
        if (off < 1e-300) break;
        for (int p = 0; p < d; p++)
            for (int q = p + 1; q < d; q++) {
                if (a[p][q] == 0.0) continue;
                double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < d; k++) {
                    double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < d; k++) {
                    double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
            }
    }
    for (int i = 0; i < d; i++) ev[i] = a[i][i];
}

/* c_A = min over points of lambda_min(A), C_A = max of lambda_max (eq:A). */
int orc_spectral_bounds(int d, long npts, const double* A, double* cA, double* CA)
{
    double lo = INFINITY, hi = -INFINITY;
    for (long p = 0; p < npts; p++) {
        double ev[3];
        sym_eig(d, A + p * d * d, ev);
        for (int i = 0; i < d; i++) {
            if (ev[i] < lo) lo = ev[i];
            if (ev[i] > hi) hi = ev[i];
        }
    }
    *cA = lo;
    *CA = hi;
    return ORC_OK;
}

/* Solve the d x d system M u = v by Gaussian elimination with partial pivoting. */
static void small_solve(int d, const double* Min, const double* v, double* u)
{
    double m[3][4];
    for (int i = 0; i < d; i++) {
        for (int j = 0; j < d; j++) m[i][j] = Min[i * d + j];
        m[i][d] = v[i];
    }
    for (int c = 0; c < d; c++) {
        int piv = c;
        for (int r = c + 1; r < d; r++)
            if (fabs(m[r][c]) > fabs(m[piv][c])) piv = r;
        if (piv != c)
            for (int j = 0; j <= d; j++) {
                double t = m[c][j];
                m[c][j] = m[piv][j];
                m[piv][j] = t;
            }
        for (int r = c + 1; r < d; r++) {
            double f = m[r][c] / m[c][c];
            for (int j = c; j <= d; j++) m[r][j] -= f * m[c][j];
        }
    }
    for (int i = d - 1; i >= 0; i--) {
        double s = m[i][d];
        for (int j = i + 1; j < d; j++) s -= m[i][j] * u[j];
        u[i] = s / m[i][i];
    }
}

/* ---------------------------------------------------------------------------------------- */
/* Inner products (Notation paragraph) and energies (eq:ev_bounds).                           */
/* ---------------------------------------------------------------------------------------- */

static double dot2(long n, const double* a, const double* b, long gsize)
{
    double s = 0.0;
    for (long i = 0; i < n; i++) s += a[i] * b[i];
    return s / (double)gsize;
}

/* (A (E_i + e_i), E_j + e_j)_2 on the integration grid. */
int orc_bilinear(int d, const int* N, int rule, const double* A, const double* Ei, const double* ei,
                 const double* Ej, const double* ej, double* out)
{
    grid_t g;
    if (op_grid(d, N, rule, &g)) return ORC_E_INVALID;
    const long S = g.size;
    double* u = (double*)malloc(sizeof(double) * d * S);
    double* v = (double*)malloc(sizeof(double) * d * S);
    double* z = (double*)malloc(sizeof(double) * d * S);
    for (int a = 0; a < d; a++)
        for (long p = 0; p < S; p++) {
            u[a * S + p] = Ei[a] + (ei ? ei[a * S + p] : 0.0);
            v[a * S + p] = Ej[a] + (ej ? ej[a * S + p] : 0.0);
        }
    pointwise_A(&g, A, u, z);
    *out = dot2((long)d * S, z, v, S);
    free(u);
    free(v);
    free(z);
    return ORC_OK;
}

/* Flux average <A (E + e)> (one column of A_H for the load E). */
int orc_flux(int d, const int* N, int rule, const double* A, const double* E, const double* e, double* flux)
{
    grid_t g;
    if (op_grid(d, N, rule, &g)) return ORC_E_INVALID;
    const long S = g.size;
    double* u = (double*)calloc((size_t)d * S, sizeof(double));
    double* z = (double*)malloc(sizeof(double) * d * S);
    for (int a = 0; a < d; a++)
        for (long p = 0; p < S; p++) u[a * S + p] = E[a] + (e ? e[a * S + p] : 0.0);
    pointwise_A(&g, A, u, z);
    for (int a = 0; a < d; a++) {
        double s = 0.0;
        for (long p = 0; p < S; p++) s += z[a * S + p];
        flux[a] = s / (double)S;
    }
    free(u);
    free(z);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------- */
/* Solvers (Sec. 3, Algorithms 1-4).                                                          */
/* ---------------------------------------------------------------------------------------- */

/* Inputs: the operator (d, N, rule, A on the integration grid), the load E, the solver, the
 * spectral bounds c_A <= C_A, the tolerance eps and an iteration cap.  If fixed_iters > 0 the
 * stopping test is ignored and exactly fixed_iters loop bodies run (iterate-matched parity).
 * Outputs: e [d][grid] (the fluctuation; for Eyre-Milton x_m - E), the number m of loop bodies
 * executed, res_hist[0..m] (the quantity of the stopping test at each step, divided by its
 * threshold scale: ||r_m||/||b|| for CG/Chebyshev, ||x_m - x_{m-1}||/||E|| for Richardson and
 * Eyre-Milton; entry 0 is 1 for the latter two), optionally energy_hist[0..m] = the energy
 * (A(E+x_m), E+x_m)_2 on the integration grid, and rel_res_true = ||b - C x||/||b|| at exit
 * (for Eyre-Milton computed for the fluctuation x - E). */
int orc_solve(int d, const int* N, int rule, const double* A, const double* E, int solver,
              double cA, double CA, double eps, int max_iter, int fixed_iters, double* e_out,
              int* iters_out, double* res_hist, double* energy_hist, double* rel_res_true)
{
    grid_t g;
    if (op_grid(d, N, rule, &g)) return ORC_E_INVALID;
    if (!(cA > 0.0) || !(CA >= cA)) return ORC_E_INVALID;
    const long S = g.size, L = (long)d * S;
    const int* band = (rule == ORC_GA) ? N : NULL;
    double normE = 0.0;
    for (int a = 0; a < d; a++) normE += E[a] * E[a];
    normE = sqrt(normE); /* ||E_N||_2 of a constant field = |E| under the 1/|grid| product */

    double* x = (double*)calloc(L, sizeof(double));
    double* b = (double*)calloc(L, sizeof(double));
    double* r = (double*)calloc(L, sizeof(double));
    double* p = (double*)calloc(L, sizeof(double));
    double* q = (double*)calloc(L, sizeof(double));
    double* t = (double*)calloc(L, sizeof(double));
    double* Ef = (double*)calloc(L, sizeof(double));
    for (int a = 0; a < d; a++)
        for (long i = 0; i < S; i++) Ef[a * S + i] = E[a];

    /* b = -G A E (eq:linsys) */
    pointwise_A(&g, A, Ef, t);
    const double normAE = sqrt(dot2(L, t, t, S));
    spectral_op(&g, band, t, b, 0);
    for (long i = 0; i < L; i++) b[i] = -b[i];
    const double normb = sqrt(dot2(L, b, b, S));
    /* A right-hand side that vanishes in exact arithmetic (homogeneous medium, load along the
     * layers of a laminate) comes out of the transforms as round-off.  It is taken as zero when
     * ||b|| <= ZERO_RHS ||A E||; CG and Chebyshev then return x = 0 before the first body. */
    const double ZERO_RHS = 1e-12;
    const int zero_rhs = !(normb > ZERO_RHS * normAE);

    int m = 0, status = ORC_OK;
    const int limit = fixed_iters > 0 ? fixed_iters : max_iter;
#define ENERGY_AT(xvec)                                                                              \
    do {                                                                                             \
        if (energy_hist) {                                                                           \
            double en_;                                                                              \
            orc_bilinear(d, N, rule, A, E, (xvec), E, (xvec), &en_);                                 \
            energy_hist[m] = en_;                                                                    \
        }                                                                                            \
    } while (0)

    if (solver == ORC_RICHARDSON) {
        /* Alg. 1 is the stationary iteration x_m = x_{m-1} + w (b - C x_{m-1}) with
         * w = 2/(c_A + C_A) from x_0 = 0 (eq:optimal_richard): the step is w times the residual,
         * and the loop ends once that step is small, ||x_m - x_{m-1}||_2 <= eps |E|. */
        const double omega = 2.0 / (cA + CA);
        res_hist[0] = 1.0;
        ENERGY_AT(x);
        while (m < limit) {
            pointwise_A(&g, A, x, t);
            spectral_op(&g, band, t, q, 0); /* q = C x */
            double ss = 0.0;
            for (long i = 0; i < L; i++) {
                const double s = omega * (b[i] - q[i]);
                x[i] += s;
                ss += s * s;
            }
            m++;
            double step = sqrt(ss / (double)S);
            res_hist[m] = normE > 0 ? step / normE : step;
            ENERGY_AT(x);
            if (!isfinite(step)) { status = ORC_E_DIVERGED; break; }
            if (fixed_iters <= 0 && step <= eps * normE) break;
        }
    } else if (solver == ORC_CG) {
        /* Alg. 2 is the Hestenes-Stiefel conjugate-gradient recurrence; x_0 = 0, r_0 = b, p_0 = r_0. */
        for (long i = 0; i < L; i++) { r[i] = b[i]; p[i] = b[i]; }
        double rr = dot2(L, r, r, S);
        res_hist[0] = zero_rhs ? 0.0 : 1.0;
        ENERGY_AT(x);
        if (!zero_rhs && (fixed_iters > 0 || sqrt(rr) > eps * normb)) {
            while (m < limit) {
                pointwise_A(&g, A, p, t);
                spectral_op(&g, band, t, q, 0); /* q = C p */
                double qp = dot2(L, q, p, S);
                double alpha = rr / qp;
                for (long i = 0; i < L; i++) {
                    x[i] += alpha * p[i];
                    r[i] -= alpha * q[i];
                }
                double rr_new = dot2(L, r, r, S);
                m++;
                res_hist[m] = sqrt(rr_new) / normb;
                ENERGY_AT(x);
                if (!isfinite(rr_new)) { status = ORC_E_DIVERGED; break; }
                if (fixed_iters <= 0 && sqrt(rr_new) <= eps * normb) break;
                double beta = rr_new / rr;
                for (long i = 0; i < L; i++) p[i] = r[i] + beta * p[i];
                rr = rr_new;
            }
        }
    } else if (solver == ORC_CHEBYSHEV) {
        /* Alg. 3 is Chebyshev semi-iteration on [c_A, C_A]: the residual after m bodies is
         * r_m = P_m(C) b with the scaled Chebyshev polynomial
         *     P_m(t) = T_m((delta - t)/c) / T_m(delta/c),  delta = (c_A + C_A)/2,  c = (C_A - c_A)/2
         * (delta is the paper's d).  Here it is built from the three-term recurrence of T_m in
         * correction form: x_{m+1} = x_m + d_m, r_{m+1} = r_m - C d_m, with
         *     d_0 = r_0 / delta,
         *     d_m = rho_m rho_{m-1} d_{m-1} + 2 rho_m / c r_m,   rho_m = T_m(s)/T_{m+1}(s),  s = delta/c,
         * and T_{m+1}(s) = 2 s T_m(s) - T_{m-1}(s) gives rho_0 = 1/s, rho_m = 1/(2 s - rho_{m-1}).
         * With k_m = c rho_m the coefficients stay finite for a one-point interval (c = 0, where
         * the method is Richardson with step 1/delta):
         *     k_0 = c^2 / delta,  D_m = 2 delta - k_{m-1} = c / rho_m,  k_m = c^2 / D_m,
         *     d_m = (k_{m-1} / D_m) d_{m-1} + (2 / D_m) r_m. */
        const double c = 0.5 * (CA - cA), delta = 0.5 * (cA + CA);
        double k = c * c / delta;
        double* dv = p;
        for (long i = 0; i < L; i++) { r[i] = b[i]; dv[i] = b[i] / delta; }
        res_hist[0] = zero_rhs ? 0.0 : 1.0;
        ENERGY_AT(x);
        if (!zero_rhs && (fixed_iters > 0 || sqrt(dot2(L, r, r, S)) > eps * normb)) {
            while (m < limit) {
                pointwise_A(&g, A, dv, t);
                spectral_op(&g, band, t, q, 0); /* q = C d_m */
                for (long i = 0; i < L; i++) {
                    x[i] += dv[i];
                    r[i] -= q[i];
                }
                double rr = dot2(L, r, r, S);
                m++;
                res_hist[m] = sqrt(rr) / normb;
                ENERGY_AT(x);
                if (!isfinite(rr)) { status = ORC_E_DIVERGED; break; }
                if (fixed_iters <= 0 && sqrt(rr) <= eps * normb) break;
                const double D = 2.0 * delta - k; /* c / rho_m */
                const double keep = k / D, gain = 2.0 / D;
                for (long i = 0; i < L; i++) dv[i] = keep * dv[i] + gain * r[i];
                k = c * c / D;
            }
        }
    } else if (solver == ORC_EYRE_MILTON) {
        /* Alg. 4 with the mean source of sign +:
         *   x_m = (A + w I)^{-1} [ F^{-1} (I - 2 G^) F (A - w I) x_{m-1} + 2 w E ],  x_0 = E,
         * w = sqrt(c_A C_A).  The fluctuation returned is x_m - E. */
        const double omega = sqrt(cA * CA);
        for (long i = 0; i < L; i++) x[i] = Ef[i];
        res_hist[0] = 1.0;
        if (energy_hist) {
            double en;
            orc_bilinear(d, N, rule, A, E, NULL, E, NULL, &en);
            energy_hist[0] = en;
        }
        double Ap[9];
        while (m < limit) {
            /* t = (A - w I) x */
            for (long i = 0; i < S; i++)
                for (int a = 0; a < d; a++) {
                    double s = -omega * x[a * S + i];
                    for (int bb = 0; bb < d; bb++) s += A[(i * d + a) * d + bb] * x[bb * S + i];
                    t[a * S + i] = s;
                }
            spectral_op(&g, band, t, q, 1); /* q = F^{-1}(I - 2G^)F t */
            double ss = 0.0;
            for (long i = 0; i < S; i++) {
                double v[3], u[3];
                for (int a = 0; a < d; a++) {
                    v[a] = q[a * S + i] + 2.0 * omega * E[a];
                    for (int bb = 0; bb < d; bb++) {
                        Ap[a * d + bb] = A[(i * d + a) * d + bb] + (a == bb ? omega : 0.0);
                    }
                }
                small_solve(d, Ap, v, u);
                for (int a = 0; a < d; a++) {
                    double s = u[a] - x[a * S + i];
                    ss += s * s;
                    x[a * S + i] = u[a];
                }
            }
            m++;
            double step = sqrt(ss / (double)S);
            res_hist[m] = normE > 0 ? step / normE : step;
            if (energy_hist) {
                for (long i = 0; i < L; i++) t[i] = x[i] - Ef[i];
                double en;
                orc_bilinear(d, N, rule, A, E, t, E, t, &en);
                energy_hist[m] = en;
            }
            if (!isfinite(step) || step > 1e12 * (normE > 0 ? normE : 1.0)) { status = ORC_E_DIVERGED; break; }
            if (fixed_iters <= 0 && step <= eps * normE) break;
        }
        for (long i = 0; i < L; i++) x[i] -= Ef[i];
    } else {
        status = ORC_E_INVALID;
    }
#undef ENERGY_AT

    if (status == ORC_OK && fixed_iters <= 0 && m >= max_iter) {
        /* the loop hit the cap without meeting its test */
        if (!(res_hist[m] <= eps)) status = ORC_E_NO_CONVERGENCE;
    }

    /* true relative residual ||b - C x|| / ||b|| */
    if (rel_res_true) {
        pointwise_A(&g, A, x, t);
        spectral_op(&g, band, t, q, 0);
        double rr = 0.0;
        for (long i = 0; i < L; i++) {
            double v = b[i] - q[i];
            rr += v * v;
        }
        rr = sqrt(rr / (double)S);
        *rel_res_true = normb > 0 ? rr / normb : rr;
    }
    memcpy(e_out, x, sizeof(double) * L);
    *iters_out = m;
    free(x); free(b); free(r); free(p); free(q); free(t); free(Ef);
    return status;
}

/* Number of threads the oracle runs with (for reporting the CPU baseline). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
