// fgh_internal.hpp -- structures shared by the host driver and the gfx950 kernels of libfgh.
//
// Operator y = G A x (eq:linsys) on a grid of L[a] points per axis with a band of B[a]
// frequencies kept per axis (eq:discrete_proj): GaNi has L = B = N, Ga has L = 2N-1, B = N.
// The transform is split into passes, one axis per pass, each pass one HBM round trip:
//
//   first   real rows along the last axis: z = A(x) op x, two real rows packed into one complex
//           row, forward FFT, split into half spectra, keep k in [0, Hb), Hb = (B_last + 1)/2
//   axis    (3D) strided forward FFT along axis 1, keep the band B1
//   middle  strided FFT along axis 0 with all d components of a frequency in one workgroup:
//           forward, keep the band B0, Fourier multiplier (G^, or I - 2G^), inverse
//   axis    (3D) strided inverse FFT along axis 1 from the band back to L1 points
//   last    half spectra back to real rows (inverse), fused solver epilogue
//
// Spectrum layouts (complex, component-major):
//   S1 [d][rows][Hb]           rows = prod_{a<d-1} L[a]           (after first / before last)
//   S2 [d][L0][B1][Hb]         3D only, after the forward axis-1 pass (middle works in place)
#pragma once
#include <stdint.h>

namespace fgh {

constexpr int kMaxRadices = 16;
constexpr int kMaxPhases = 16;
constexpr int kThreads = 256;

// One FFT length: its Stockham radix sequence and where its twiddle table starts.
struct Axis {
    int L;
    int nst;
    int rad[kMaxRadices];
    int tw;  // offset (complex elements) of exp(-2 pi i m / L), m in [0, L), in the table buffer
};

struct Geo {
    int d;
    int L[3];
    int B[3];
    int Hb;             // (B[d-1] + 1) / 2
    long long npts;     // prod L
    long long rows;     // npts / L[d-1]
    long long s1;       // rows * Hb               (complex elements per component of S1)
    long long s2;       // L0 * B1 * Hb (3D), s1 (2D)
    int cols_mid;       // columns of the middle pass: B1 * Hb (3D), Hb (2D)
};

// Coefficient representation seen by the pass kernels.
enum AKind : int { AK_SYM = 0, AK_ISO = 1, AK_PHASE = 2 };

// What the first pass computes before its FFT.
enum FirstOp : int {
    OP_AX = 0,      // z = A (x + E)   (E may be zero)
    OP_E = 1,       // z = A E         (no vector read: the right-hand side)
    OP_EM = 2,      // z = (A - w I) x (Eyre-Milton)
    OP_ID = 3,      // z = x           (the projection alone)
    OP_AP_CG = 4    // p <- r + beta p (beta from the device scalars), write p, z = A p
};

// Fourier multiplier of the middle pass.
enum Mult : int { MULT_G = 0, MULT_EM = 1 };

// Solver epilogue of the last pass.
enum Epi : int {
    EPI_STORE = 0,  // y = s * (G A x); acc += y.y
    EPI_RICH = 1,   // step = -w (G A (E + x)); x += step; acc += step.step
    EPI_CG = 2,     // q = G A p; acc += q.p
    EPI_CHEB = 3,   // r -= alpha q; x += alpha p; p = r - beta p; acc += r.r
    EPI_EM = 4      // x_new = (A + wI)^{-1} (y + 2 w E); acc += |x_new - x|^2; x = x_new
};

// Device-resident solver state.  The loop kernels of an iteration return at once when done != 0,
// so the host can enqueue iterations in chunks and synchronise once per chunk: iterations after
// the stopping test fired are no-ops and the count m stays exact.
struct Scalars {
    double rr;          // (r, r) of the current residual (raw sum over the grid)
    double rr_new;
    double qp;          // (C p, p)
    double alpha;
    double beta;
    double total;       // last reduced value
    double thr;         // stop when sqrt(value / npts) <= thr (value: (r,r) or |step|^2); < 0: never
    double npts;
    double blowup;      // diverged when sqrt(value / npts) > blowup (0: only non-finite values)
    double cheb_c, cheb_delta;  // Chebyshev interval half-width and centre
    double last;        // the stopping-test quantity sqrt(value / npts) of the last body
    int done;           // 0 running, 1 stopping test met, 2 iteration cap, 3 diverged
    int m;              // loop bodies executed
    int limit;          // cap on m
    int pend_n;         // partial sums of a loop reduction deferred to the next body (0: none)
    int pend_op;        //   and its RedOp
    double aux[40];     // [0, 16): loads for fgh_effective; [16, 40): multi-value reductions
};

enum RedOp : int {
    RED_TOTAL = 0,     // total -> s.total
    RED_CG_ALPHA = 1,  // s.qp = total; s.alpha = s.rr / s.qp
    RED_CG_END = 2,    // s.rr_new = total; s.beta = s.rr_new / s.rr; s.rr = s.rr_new; end of a body
    RED_SET_RR = 3,    // s.rr = total
    RED_STEP_END = 4,  // total = |step|^2 (Richardson, Eyre-Milton); end of a body
    RED_CHEB_END = 5   // total = (r, r); end of a body; next alpha, beta of Algorithm 3
};

struct CoefArgs {
    int kind;                 // AKind
    int ncoef;                // 3 (2D) / 6 (3D) for AK_SYM, 1 for AK_ISO
    const void* coef;         // AK_SYM [ncoef][npts] / AK_ISO [npts], element type of the pass
    const uint8_t* phase;     // AK_PHASE [npts]
    double tab[kMaxPhases][6];     // AK_PHASE packed symmetric per phase
    double tab_inv[kMaxPhases][6]; // AK_PHASE packed (A + w I)^{-1} per phase (Eyre-Milton)
};

}  // namespace fgh
