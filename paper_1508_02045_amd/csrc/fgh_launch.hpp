// fgh_launch.hpp -- host-side launch wrappers of the libfgh kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "fgh_args.hpp"
#include "fgh_internal.hpp"

namespace fgh {

// Per-pass device timing: launches bracketed by HIP events on the plan's stream.
enum PassKind : int {
    PK_FIRST = 0, PK_AXIS_FWD = 1, PK_MIDDLE = 2, PK_AXIS_INV = 3, PK_LAST = 4,
    PK_CG_UPDATE = 5,  // CG's x += alpha p, r -= alpha q, (r, r) partial sums
    PK_REDUCE = 6,     // single-workgroup loop reductions
    PK_KINDS = 7
};
// Events for the next pass launch while a pass is being timed: the launch takes them as the
// start and stop events of the dispatch itself (hipExtLaunchKernelGGL), so the measured time is
// the kernel's own execution time.
struct PassEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local PassEvents g_pass_events;

struct Profiler {
    static constexpr int kPool = 256;
    hipEvent_t ev[2 * kPool];
    int kind[kPool];
    int used = 0;
    bool ready = false;
    double ms[PK_KINDS] = {};
    long long n[PK_KINDS] = {};
    std::vector<float> dur[PK_KINDS];  // every timed launch (ms), for the working-launch totals
    hipStream_t stream = nullptr;
    unsigned mask = 0u;  // pass kinds timed (bit k: PassKind k)
    bool wants(int k) const { return (mask >> k) & 1u; }
    hipError_t init(hipStream_t s);
    void destroy();
    hipError_t begin(int k);
    hipError_t end();
    hipError_t drain();
    // Totals over the launches that did work: a launch of a solver body after the loop has
    // stopped returns at once; launches shorter than 30 % of the kind's median are left out.
    void working(int k, double* ms_out, long long* n_out) const;
};

// Everything one operator application needs (one precision).
struct OpPlan {
    Geo g;
    Axis ax[3];              // FFT descriptor per axis (length L[a])
    const void* tw[3];       // device twiddle table per axis (element type of the pass)
    void* SA;                // spectrum buffers (complex, element type of the pass)
    void* SB;
    CoefArgs A;              // coefficients as seen by the passes
    int rpb, npen;           // first/last passes: rows per block, complex pencils per block
    int rpb_first;           // the specialised first pass: rows per block (even; tuned)
    int P_axis, P_mid;       // axis / middle passes: tile width
    int mid_pad;             // specialised middle pass: LDS column stride L + mid_pad (tuned)
    size_t lds_first, lds_axis, lds_mid;
    size_t lds_first_v2;     // the specialised first pass (one row buffer)
    int rpb_first_x;         // the same for CG's first pass with the deferred iterate update (tuned)
    size_t lds_first_x;
    size_t lds_last_v2;      // the specialised last pass (one row buffer)
    int rpb_fused;           // the fused last + first pass: rows per block (even or the last pass's; tuned)
    size_t lds_fused;        //   and its LDS (one row buffer, two coefficient tables)
    bool v2_row, v2_axis, v2_mid;  // size-specialised kernels for the row / axis-1 / axis-0 passes
    double* partials;        // one double per block of the last pass (and of vector kernels)
    Scalars* sc;
    hipStream_t stream;
    Profiler* prof = nullptr;  // non-null while profiling is enabled
};

// Parameters of one application: what the first pass reads, the multiplier, the epilogue.
struct ApplyArgs {
    int op = OP_AX;          // FirstOp
    int mult = MULT_G;       // Mult
    int epi = EPI_STORE;     // Epi
    const void* x = nullptr; // first-pass input vector ([d][npts])
    void* p_cg = nullptr;    // OP_AP_CG: p (updated in place)
    const void* r_cg = nullptr;
    void* x_cg = nullptr;    // OP_AP_CG: x += alpha p before p is replaced (the previous body's update)
    double E[3] = {0, 0, 0};
    double omega = 0.0;      // Eyre-Milton omega, Richardson omega
    double alpha = 0.0, beta = 0.0, sgn = 1.0;
    void* y = nullptr;       // EPI_STORE output
    void* ex = nullptr;      // epilogue vectors
    void* er = nullptr;
    void* ep = nullptr;
    void* eq = nullptr;
    const void* src = nullptr; // EPI_EM: additive source field (refinement); nullptr: 2 w E
    bool loop = false;       // part of a solver loop: kernels skip work once the stop flag is set
    bool cheb_dev = false;   // Chebyshev alpha, beta from the device scalars
    // Fused loops (specialised row kernels, epilogues RICH / CHEB / EM): the last pass also runs
    // the next body's first pass with operator next_op on the updated vector; the next body then
    // skips its first pass.  first_only runs the first pass alone (the loop's prologue).
    int next_op = -1;
    bool skip_first = false;
    bool first_only = false;
    // >= 0 (3D, specialised row and axis kernels): the loop reduction (RedOp) of this body's last
    // pass is left to the first workgroup of the next body's forward axis pass, which replaces
    // the separate single-block reduction launch
    int defer_redop = -1;
};

// Whether the plan's last pass can run the next body's first pass (see ApplyArgs::next_op).
inline bool fusable(const OpPlan& op) { return op.v2_row; }

template <typename T>
hipError_t run_apply(const OpPlan& op, const ApplyArgs& a, int* nblocks_last);

// ------------------------------------------------------------------------------------------
// Several plans of one shape in shared launches ("members" of a batch).  Each member keeps its
// own buffers, coefficients, loop scalars and partial sums; a batched launch runs the same pass
// for every member, one grid row (or plane) per member, with the member's argument block read
// from a device table.  A member's workgroups see the block ids of the single-plan launch, so its
// tile mapping, partial sums and summation order -- hence its results -- are those of the plan
// alone.  Only the size-specialised passes are batched.
// ------------------------------------------------------------------------------------------
// The argument blocks of one application, built exactly as the single-plan launch builds them.
template <typename T>
struct ApplyBundle {
    FirstArgs<T> fa;
    AxisArgs<T> xf, xi;      // forward and inverse strided passes (3D)
    MidArgs<T> ma;
    LastArgs<T> la;
    unsigned nblk1, nblk_last;
    int op, mult, epi;
    bool fused, skip_first, first_only;
};
struct ReduceArgs {
    const double* partials;
    int n;
    Scalars* sc;
};
template <typename T>
struct UpdateArgs {
    long long n;
    T* x;
    T* r;
    const T* p;
    const T* q;
    const Scalars* sc;
    double* partials;
};
// Device tables of a batch of up to kMaxBatch members, carved out of a device region of
// kBatchSlabBytes (struct-of-arrays: the argument blocks of one kind are contiguous).
constexpr int kMaxBatch = 8;
constexpr size_t kBatchSlabBytes = 64 * 1024;
template <typename T>
struct BatchTables {
    FirstArgs<T>* fa;
    AxisArgs<T>* xf;
    AxisArgs<T>* xi;
    MidArgs<T>* ma;
    LastArgs<T>* la;
    ReduceArgs* red;   // loop reductions of the last pass's partial sums
    ReduceArgs* red2;  // loop reductions of the CG update's partial sums
    UpdateArgs<T>* upd;
    size_t bytes;      // bytes used from the start of the region
};
template <typename T>
BatchTables<T> batch_tables(void* region);
// The argument blocks of application `a` on plan `op` (no launch).
template <typename T>
hipError_t build_bundle(const OpPlan& op, const ApplyArgs& a, ApplyBundle<T>* out);
// Whether plans of this shape can share launches (size-specialised passes throughout).
bool batchable(const OpPlan& op);
// One application per member from the uploaded tables; op0 is any member's plan (shared launch
// configuration), b0 its bundle (shared flags and tile counts), nb the member count.
template <typename T>
hipError_t run_apply_batch(const OpPlan& op0, const ApplyBundle<T>& b0, const BatchTables<T>& t, int nb);
hipError_t run_reduce_batch(hipStream_t s, const ReduceArgs* tab, int nb, int redop);
template <typename T>
hipError_t run_cg_update_batch(hipStream_t s, const UpdateArgs<T>* tab, int nb);

hipError_t run_reduce(const OpPlan& op, int n, int redop, double* host_out);

// The middle pass alone on the plan's spectrum buffer (tile-width tuning at plan creation; the
// buffer's contents are overwritten).
template <typename T>
hipError_t run_middle_only(const OpPlan& op);

// The forward axis-1 pass alone (3D) from the first into the second spectrum buffer (tile-width
// tuning at plan creation; the second buffer's contents are overwritten).
template <typename T>
hipError_t run_axis_only(const OpPlan& op);

// The first pass alone (identity operator) from the vector x into the plan's first spectrum
// buffer (tile tuning at plan creation).
template <typename T>
hipError_t run_first_only(const OpPlan& op, const T* x);

// The fused last + first Richardson pass alone, with step 0 (x is read and rewritten unchanged),
// on the plan's first spectrum buffer (tile tuning at plan creation; the buffer is overwritten).
template <typename T>
hipError_t run_fused_only(const OpPlan& op, T* x);

// Trigonometric prolongation of a real vector field from the N grid of `opn` to the 2N-1 grid of
// `opm` (both double precision; opm's spectrum buffers are used as scratch).
hipError_t run_prolong(const OpPlan& opn, const OpPlan& opm, const double* xn, double* ym);
hipError_t run_reduce_async(const OpPlan& op, int n, int redop);
hipError_t run_set_scalar(const OpPlan& op, double* dst, double v);
hipError_t run_init_loop(const OpPlan& op, double rr, double alpha, double beta, double thr, double npts,
                         double blowup, double cheb_c, double cheb_delta, int limit);

int vec_blocks();
template <typename T>
hipError_t run_cg_update(const OpPlan& op, long long n, T* x, T* r, const T* p, const T* q);
template <typename T>
hipError_t run_cg_x(const OpPlan& op, long long n, T* x, const T* p);
// CG's first pass with the deferred iterate update alone (tile timing): x += alpha p,
// p = r + beta p, A p into SA
template <typename T>
hipError_t run_first_cg_only(const OpPlan& op, T* x, const T* r, T* p);
template <typename T>
hipError_t run_fill(hipStream_t s, long long n, T* x, T v);
template <typename T>
hipError_t run_fill_field(hipStream_t s, int d, long long npts, T* x, const double* v);
template <typename T>
hipError_t run_copy(hipStream_t s, long long n, T* dst, const T* src);
hipError_t run_f64_to_f32(hipStream_t s, long long n, float* dst, const double* src);
hipError_t run_add_f32_to_f64(hipStream_t s, long long n, double* x, const float* d);
hipError_t run_add_f64(hipStream_t s, long long n, double* x, const double* d);
hipError_t run_axpby(hipStream_t s, long long n, double* y, double a, const double* x, double b);
// Twiddle table exp(-2 pi i m / L), m in [0, L), computed on the device (FP64).
hipError_t run_twiddles(hipStream_t s, int L, double2* tw);
hipError_t run_norm_AE(const OpPlan& op, const double* E, int* nblocks);
template <typename T>
hipError_t run_dot(const OpPlan& op, long long n, const T* a, const T* b, int* nblocks);

// Effective quantities: partials [nblocks][nrhs*nrhs + nrhs*d].
hipError_t run_effective(const OpPlan& op, int nrhs, const double* E, const double* e, int* nblocks);
// History entries of the non-conformity of the iterate x (Sec. 4.4): ||G x - (x - shift)|| and
// |<x> - shift|; y receives G x (a vector of the integration grid); uses the partial sums.
hipError_t run_hist_nonconf(const OpPlan& op, const double* x, const double* shift, double* y, double* nc,
                            double* mean, int cap);
// History entry of a solver loop (stopping-test quantity, energy from k_effective partial sums).
hipError_t run_hist(hipStream_t stream, const double* partials, int nb, int nvals, const Scalars* sc, double* res,
                    double* en, int cap, double en_scale);
hipError_t run_reduce_multi(const OpPlan& op, int nblocks, int nvals, double* host_out);

// Coefficient preparation.
hipError_t run_to_f32(hipStream_t s, long long n, float* dst, const double* src);
hipError_t run_eig_bounds(hipStream_t s, int d, int kind, const double* coef, long long npts,
                          double* partials, int* nblocks);
hipError_t run_minmax_reduce(hipStream_t s, const double* partials, int nblocks, double* host_lo_hi);
hipError_t run_phase_mask(hipStream_t s, const uint8_t* phase, long long npts, unsigned* mask);

// Ga coefficients on the double grid from a pixel-wise constant field on the N grid.
struct GaAsm {
    int d;
    int N[3], M[3];
    long long nN, nM;
    const double2* twN[3];   // exp(-2 pi i m / N_a)
    const double2* twM[3];   // exp(-2 pi i m / M_a)
    const double* sinc[3];   // sinc(n / N_a) for the M_a positions of axis a
    double2* c0;             // scratch complex buffers, |M| elements each
    double2* c1;
};
hipError_t run_ga_component(hipStream_t s, const GaAsm& ga, int kind, const double* coef, int comp,
                            const uint8_t* phase, const double* phase_vals, int nphase,
                            double* out /* [nM] */);

}  // namespace fgh
