// fgh_api.cpp -- host side of libfgh: plans, workspace layout, coefficient set-up and the
// solver drivers of Algorithms 1-4 (Sec. 3) on top of the gfx950 passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/fgh.h"
#include "fgh_internal.hpp"
#include "fgh_launch.hpp"
#include "fgh_v2.hpp"
#include "fgh_batch.hpp"

using namespace fgh;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kLdsBudgetDefault = 80 * 1024;

// LDS bytes per workgroup the launch configuration may use (tuning knob: FGH_LDS_BUDGET).
size_t lds_budget()
{
    const char* v = std::getenv("FGH_LDS_BUDGET");
    if (v) {
        const long b = std::atol(v);
        if (b >= 8192 && b <= 160 * 1024) return (size_t)b;
    }
    return kLdsBudgetDefault;
}
constexpr double kZeroRhs = 1e-12;      // b is taken as zero when ||b|| <= kZeroRhs ||A E||
constexpr int kMaxLanczos = 4096;       // cap on the CG steps of fgh_estimate_bounds
constexpr double kLanczosInvariant = 1e-14;  // ||r_m|| / ||b|| below which K_m is taken as invariant
constexpr double kInnerTolMin = 1e-4;   // FP32 inner solves stop at this relative residual

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int ncoef_for(int d) { return d == 2 ? 3 : 6; }

// Radix sequence of an odd length: 7s, 5s, 3s, then any other prime factor.
bool factorize(int L, Axis* ax)
{
    int n = L, k = 0;
    const int small[3] = {7, 5, 3};
    for (int p : small)
        while (n % p == 0) {
            if (k >= kMaxRadices) return false;
            ax->rad[k++] = p;
            n /= p;
        }
    for (int p = 11; n > 1; p += 2)
        while (n % p == 0) {
            if (k >= kMaxRadices) return false;
            ax->rad[k++] = p;
            n /= p;
        }
    ax->L = L;
    ax->nst = k;
    return true;
}

struct Config {
    int rpb, npen, P_axis, P_mid;
    size_t lds_first, lds_first_v2, lds_last_v2, lds_axis, lds_mid;
    bool v2_row, v2_axis, v2_mid;
};

int env_int(const char* name, int dflt)
{
    const char* v = std::getenv(name);
    if (!v) return dflt;
    const int x = std::atoi(v);
    return x > 0 ? x : dflt;
}

// The device's last-level cache (MI355X: 256 MiB of Infinity Cache).
constexpr double kLastLevelCacheBytes = 256.0 * 1024 * 1024;

// the variable's integer value, zero and negative values included (dflt when unset)
int env_int_any(const char* name, int dflt)
{
    const char* v = std::getenv(name);
    return v ? std::atoi(v) : dflt;
}

// Tile choice per pass: the largest tile whose LDS footprint fits the budget (tuning knobs:
// FGH_RPB, FGH_P_AXIS, FGH_P_MID cap the rows per block and the tile widths).  The specialised
// kernels hold one copy of the tile (plus the twiddle table); the generic ones two (ping-pong).
Config choose_config(const Geo& g, size_t cs /* bytes per complex */, size_t rs /* bytes per real */)
{
    Config c{};
    const size_t kLdsBudget = lds_budget();
    const int d = g.d;
    const int Ll = g.L[d - 1];
    const size_t tabb = kMaxPhases * 6 * rs;
    // the specialised kernels index within a vector or spectrum with 32-bit offsets
    const long long span = (long long)d * std::max(g.npts, std::max(g.s1, g.s2));
    const bool small = span < (1LL << 31);
    c.v2_row = small && v2_supported(Ll);
    c.v2_axis = small && d == 3 && v2_supported(g.L[1]);
    c.v2_mid = small && v2_supported(g.L[0]);
    c.rpb = 1;
    int rpb_cap = env_int("FGH_RPB", c.v2_row ? 8 : 32);
    if (rpb_cap > 32) rpb_cap = 32;
    for (int rpb = rpb_cap; rpb >= 1; rpb--) {
        const int npen = (rpb * d + 1) / 2;
        // specialised (in place): twiddles + npen rows of L + 1 slots + table; generic: two row
        // buffers
        const size_t lds = c.v2_row ? (size_t)(Ll + npen * (Ll + 1)) * cs + tabb
                                    : (size_t)(Ll + 2 * npen * Ll) * cs + tabb;
        if (lds <= kLdsBudget || rpb == 1) {
            c.rpb = rpb;
            c.lds_first = lds;
            // the specialised row passes work in place: twiddles + npen rows (+1 slot each in the
            // last pass) + table
            c.lds_first_v2 = (size_t)(Ll + npen * Ll) * cs + tabb;
            c.lds_last_v2 = (size_t)(Ll + npen * (Ll + 1)) * cs + tabb;
            break;
        }
    }
    c.npen = (c.rpb * d + 1) / 2;
    const int Ps[5] = {16, 8, 4, 2, 1};
    c.P_axis = 1;
    c.lds_axis = 0;
    const int pax_cap = env_int("FGH_P_AXIS", 16), pmid_cap = env_int("FGH_P_MID", 16);
    // exact tile widths (tuning): FGH_P_EXACT=1 takes FGH_P_AXIS / FGH_P_MID as given
    const bool exact = env_int("FGH_P_EXACT", 0) != 0;
    if (d == 3)
        for (int P : Ps) {
            if (exact) P = pax_cap;
            if (P > pax_cap) continue;
            const size_t lds = c.v2_axis ? (size_t)(g.L[1] + P * g.L[1]) * cs : (size_t)(g.L[1] + 2 * P * g.L[1]) * cs;
            if (lds <= kLdsBudget || P == 1) {
                c.P_axis = P;
                c.lds_axis = lds;
                break;
            }
        }
    c.P_mid = 1;
    for (int P : Ps) {
        if (exact) P = pmid_cap;
        if (P > pmid_cap) continue;
        const size_t lds = c.v2_mid ? (size_t)(g.L[0] + d * P * g.L[0]) * cs : (size_t)(g.L[0] + (d + 1) * P * g.L[0]) * cs;
        if (lds <= kLdsBudget || P == 1) {
            c.P_mid = P;
            c.lds_mid = lds;
            break;
        }
    }
    return c;
}

bool make_geo(int d, const int32_t* N, int rule, Geo* g)
{
    if (d != 2 && d != 3) return false;
    if (!N) return false;
    g->d = d;
    g->npts = 1;
    for (int a = 0; a < 3; a++) g->L[a] = g->B[a] = 1;
    for (int a = 0; a < d; a++) {
        if (N[a] < 3 || N[a] % 2 == 0 || N[a] > 8191) return false;
        g->B[a] = N[a];
        g->L[a] = rule == FGH_GA ? 2 * N[a] - 1 : N[a];
        g->npts *= g->L[a];
    }
    g->Hb = (g->B[d - 1] + 1) / 2;
    g->rows = g->npts / g->L[d - 1];
    g->s1 = g->rows * g->Hb;
    g->s2 = d == 3 ? (long long)g->L[0] * g->B[1] * g->Hb : g->s1;
    g->cols_mid = d == 3 ? g->B[1] * g->Hb : g->Hb;
    return true;
}

struct Layout {
    size_t tw64[3], tw32[3], SA, SB, vec64, vec32, partials, scalars, mask, coef64, coef32, sinc[3], twN[3], twM[3];
    size_t slab;  // argument tables of batched launches led by this plan
    size_t total;
    long long npart;
};

Layout make_layout(const Geo& g, const int32_t* N, int rule, int prec, int akind)
{
    Layout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const int d = g.d;
    for (int a = 0; a < d; a++) l.tw64[a] = take((size_t)g.L[a] * 16);
    for (int a = 0; a < d; a++) l.tw32[a] = take((size_t)g.L[a] * 8);
    const long long sp = g.s1 > g.s2 ? g.s1 : g.s2;
    l.SA = take((size_t)d * sp * 16);
    l.SB = take((size_t)d * sp * 16);
    const long long nv = (long long)d * g.npts;
    // three double vectors (CG r, p, q; Chebyshev r, p; refinement r, delta, G delta), which
    // also host the Ga-assembly scratch at set-up time
    size_t v64 = (size_t)3 * nv * 8;
    long long nM = 1, nN = 1;
    for (int a = 0; a < d; a++) {
        nN *= N[a];
        nM *= 2 * N[a] - 1;
    }
    if (rule == FGH_GA && v64 < (size_t)2 * nM * 16) v64 = (size_t)2 * nM * 16;
    // and a third spectrum for the middle pass's tile timing
    if (v64 < (size_t)d * sp * 16) v64 = (size_t)d * sp * 16;
    l.vec64 = take(v64);
    l.vec32 = take(prec == FGH_FP32_REFINED ? (size_t)4 * nv * 4 : 0);
    const Config c64 = choose_config(g, 16, 8);
    const Config c32 = choose_config(g, 8, 4);
    long long nb = (g.rows + c64.rpb - 1) / c64.rpb;
    const long long nb32 = (g.rows + c32.rpb - 1) / c32.rpb;
    if (nb32 > nb) nb = nb32;
    long long np = nb;
    if (np < 1024 * 2 + 2) np = 1024 * 2 + 2;
    if (np < 512 * 18) np = 512 * 18;
    l.npart = np + 64;
    l.partials = take((size_t)l.npart * 8);
    l.scalars = take(sizeof(Scalars));
    l.slab = take(kBatchSlabBytes);
    l.mask = take(16);
    const int ncoef_op = (akind == FGH_A_SYM) ? ncoef_for(d) : 1;
    l.coef64 = take(rule == FGH_GA ? (size_t)ncoef_op * g.npts * 8 : 0);
    const bool need32 = prec == FGH_FP32_REFINED && (rule == FGH_GA || akind != FGH_A_PHASE);
    l.coef32 = take(need32 ? (size_t)ncoef_op * g.npts * 4 : 0);
    for (int a = 0; a < d; a++) {
        l.sinc[a] = take(rule == FGH_GA ? (size_t)(2 * N[a] - 1) * 8 : 0);
        l.twN[a] = take(rule == FGH_GA ? (size_t)N[a] * 16 : 0);
        l.twM[a] = take(rule == FGH_GA ? (size_t)(2 * N[a] - 1) * 16 : 0);
    }
    l.total = off;
    return l;
}

// Eigenvalues of a packed symmetric 2x2 / 3x3 block on the host (cyclic Jacobi).
void host_sym_eigs(int d, const double* p, double* lo, double* hi)
{
    double a[3][3];
    if (d == 2) {
        a[0][0] = p[0]; a[0][1] = a[1][0] = p[1]; a[1][1] = p[2];
    } else {
        a[0][0] = p[0]; a[0][1] = a[1][0] = p[1]; a[0][2] = a[2][0] = p[2];
        a[1][1] = p[3]; a[1][2] = a[2][1] = p[4]; a[2][2] = p[5];
    }
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0.0;
        for (int i = 0; i < d; i++)
            for (int j = i + 1; j < d; j++) off += a[i][j] * a[i][j];
        if (off < 1e-300) break;
        for (int pp = 0; pp < d; pp++)
            for (int q = pp + 1; q < d; q++) {
                if (a[pp][q] == 0.0) continue;
                const double th = (a[q][q] - a[pp][pp]) / (2.0 * a[pp][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < d; k++) {
                    const double akp = a[k][pp], akq = a[k][q];
                    a[k][pp] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < d; k++) {
                    const double apk = a[pp][k], aqk = a[q][k];
                    a[pp][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
            }
    }
    *lo = 1e300;
    *hi = -1e300;
    for (int i = 0; i < d; i++) {
        *lo = std::fmin(*lo, a[i][i]);
        *hi = std::fmax(*hi, a[i][i]);
    }
}

// Packed inverse of (A + w I) for a packed symmetric block.
void host_shift_inverse(int d, const double* p, double w, double* inv)
{
    if (d == 2) {
        const double m00 = p[0] + w, m01 = p[1], m11 = p[2] + w;
        const double det = m00 * m11 - m01 * m01;
        inv[0] = m11 / det;
        inv[1] = -m01 / det;
        inv[2] = m00 / det;
    } else {
        const double m00 = p[0] + w, m01 = p[1], m02 = p[2], m11 = p[3] + w, m12 = p[4], m22 = p[5] + w;
        const double c00 = m11 * m22 - m12 * m12, c01 = m02 * m12 - m01 * m22, c02 = m01 * m12 - m02 * m11;
        const double c11 = m00 * m22 - m02 * m02, c12 = m01 * m02 - m00 * m12, c22 = m00 * m11 - m01 * m01;
        const double det = m00 * c00 + m01 * c01 + m02 * c02;
        inv[0] = c00 / det; inv[1] = c01 / det; inv[2] = c02 / det;
        inv[3] = c11 / det; inv[4] = c12 / det; inv[5] = c22 / det;
    }
}

}  // namespace

struct fgh_plan_s {
    int d;
    int32_t N[3];
    int rule, prec, akind;
    Geo g;
    Layout lay;
    char* ws;
    hipStream_t stream;
    double cA, CA;
    int nphase;
    double tab[kMaxPhases][6];
    int ncoef_op;             // 1 (scalar A_{2N-1} / iso) or ncoef
    OpPlan op64, op32;
    double* r64;
    double* p64;
    double* q64;
    float* x32;
    float* r32;
    float* p32;
    float* q32;
    double* host_buf;         // pinned host scalars
    Profiler* prof;           // per-pass timing while enabled
    hipStream_t caller;       // the caller's stream
    hipStream_t sstream;      // plan-internal stream of fgh_solve (graph capture needs one)
    hipGraph_t graph;         // captured loop bodies (reused while the key matches)
    hipGraphExec_t gexec;
    uint64_t gkey;
    // loop history (fgh_plan_set_history): device ring buffers [nrhs][hist_cap], nullptr: off
    double* hist_res;
    double* hist_en;
    double* hist_nc;                     // non-conformity ||G x - x~|| and its mean-value part
    double* hist_mean;
    double* hist_scratch;                // caller's vector for G x
    int hist_cap;
    fgh_plan hist_ga;                    // Ga plan of the GaNi bound monitor, or nullptr
    std::function<hipError_t()> hist_fn;  // records the entry of the current body count
    uint64_t hist_key;
};

namespace {

#define HIPOK(x)                                 \
    do {                                         \
        if ((x) != hipSuccess) return FGH_E_DEVICE; \
    } while (0)

fgh_status upload_twiddles(fgh_plan p)
{
    std::vector<double> t64;
    std::vector<float> t32;
    for (int a = 0; a < p->d; a++) {
        const int L = p->g.L[a];
        t64.resize(2 * (size_t)L);
        t32.resize(2 * (size_t)L);
        for (int m = 0; m < L; m++) {
            const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)L;
            const double c = (double)cosl(ang), s = -(double)sinl(ang);
            t64[2 * m] = c;
            t64[2 * m + 1] = s;
            t32[2 * m] = (float)cosl(ang);
            t32[2 * m + 1] = (float)(-sinl(ang));
        }
        HIPOK(hipMemcpyAsync(p->ws + p->lay.tw64[a], t64.data(), (size_t)L * 16, hipMemcpyHostToDevice, p->stream));
        HIPOK(hipMemcpyAsync(p->ws + p->lay.tw32[a], t32.data(), (size_t)L * 8, hipMemcpyHostToDevice, p->stream));
        HIPOK(hipStreamSynchronize(p->stream));
    }
    return FGH_OK;
}

// Operator description of one precision over given device buffers: twiddle tables per axis, the
// two half-spectrum buffers, the partial sums and the loop scalar block; static tile choices.
void fill_opplan_at(OpPlan* op, const Geo& g, bool f32, char* const tw[3], char* SA, char* SB, double* partials,
                    Scalars* sc, hipStream_t stream)
{
    const Config c = choose_config(g, f32 ? 8 : 16, f32 ? 4 : 8);
    op->g = g;
    for (int a = 0; a < 3; a++) {
        if (a < g.d) factorize(g.L[a], &op->ax[a]);
        op->ax[a].tw = 0;
        op->tw[a] = a < g.d ? tw[a] : nullptr;
    }
    op->SA = SA;
    op->SB = SB;
    op->rpb = c.rpb;
    op->rpb_first = c.rpb;
    op->mid_pad = 0;
    op->npen = c.npen;
    op->P_axis = c.P_axis;
    op->P_mid = c.P_mid;
    op->lds_first = c.lds_first;
    op->lds_first_v2 = c.lds_first_v2;
    op->rpb_first_x = c.rpb;
    op->lds_first_x = c.lds_first_v2;
    op->lds_last_v2 = c.lds_last_v2;
    op->rpb_fused = c.rpb;
    op->lds_fused = c.lds_last_v2 + kMaxPhases * 6 * (f32 ? 4 : 8);
    op->lds_axis = c.lds_axis;
    op->lds_mid = c.lds_mid;
    op->v2_row = c.v2_row;
    op->v2_axis = c.v2_axis;
    op->v2_mid = c.v2_mid;
    op->partials = partials;
    op->sc = sc;
    op->stream = stream;
}

void fill_opplan(fgh_plan p, OpPlan* op, bool f32)
{
    char* tw[3] = {nullptr, nullptr, nullptr};
    for (int a = 0; a < p->d; a++) tw[a] = p->ws + (f32 ? p->lay.tw32[a] : p->lay.tw64[a]);
    fill_opplan_at(op, p->g, f32, tw, p->ws + p->lay.SA, p->ws + p->lay.SB,
                   reinterpret_cast<double*>(p->ws + p->lay.partials), reinterpret_cast<Scalars*>(p->ws + p->lay.scalars),
                   p->stream);
}

// FGH_TUNE_LOG=1: the tuners print each candidate's time (three launches) to stderr.
void tune_log(const char* pass, bool f32, int cand, int pad, float ms)
{
    static const bool on = env_int("FGH_TUNE_LOG", 0) != 0;
    if (on) std::fprintf(stderr, "fgh tune %s %s: %d%s %.1f us\n", pass, f32 ? "fp32" : "fp64", cand, pad ? "+pad" : "", ms * 1e3f / 3);
}

// Tile width of the strided axis-1 passes (3D), measured at plan creation like the middle pass's:
// powers of two and the widths that split the Hb columns of a half-spectrum row into equal tiles
// (a ragged last tile leaves most of its workgroup idle).  The per-column arithmetic does not
// depend on the width, so results are identical whatever is chosen.
fgh_status tune_axis(fgh_plan p, OpPlan* op, bool f32)
{
    if (p->d != 3 || env_int("FGH_TUNE", 1) == 0 || env_int("FGH_P_EXACT", 0) != 0) return FGH_OK;
    static std::mutex mu;
    static std::map<std::vector<long long>, int> cache;
    const Geo& g = op->g;
    const std::vector<long long> key = {f32 ? 1 : 0, g.L[1], g.B[1], g.Hb, g.L[0], op->v2_axis ? 1 : 0};
    const size_t cs = f32 ? 8 : 16;
    const size_t L1 = (size_t)g.L[1];
    auto lds_of = [&](int P) { return op->v2_axis ? (L1 + (size_t)P * L1) * cs : (L1 + 2 * (size_t)P * L1) * cs; };
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            op->P_axis = it->second;
            op->lds_axis = lds_of(op->P_axis);
            return FGH_OK;
        }
    }
    std::vector<int> cand = {4, 8, 12, 16};
    for (int P = 6; P <= 24; P++)
        if (g.Hb % P == 0 && std::find(cand.begin(), cand.end(), P) == cand.end()) cand.push_back(P);
    hipEvent_t e0, e1;
    HIPOK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FGH_E_DEVICE;
    }
    int best = op->P_axis;
    float best_ms = 1e30f;
    void* const bufs[3] = {op->SA, op->SB, p->ws + p->lay.vec64};
    hipError_t err = hipSuccess;
    // two rounds over the candidates: the fastest single timing wins (robust to a noisy first round)
    for (int round = 0; round < 2 && err == hipSuccess; round++)
    for (int P : cand) {
        if (lds_of(P) > lds_budget() || P > g.Hb) continue;
        OpPlan o = *op;
        o.P_axis = P;
        o.lds_axis = lds_of(P);
        o.prof = nullptr;
        // launches cycle A -> B, C -> A, B -> C over the spectra and the vector storage: each reads
        // what the last-level cache has had two launches' data to drop since (see tune_middle)
        auto run_on = [&](int k) {
            OpPlan oo = o;
            oo.SA = bufs[(3 - k % 3) % 3];
            oo.SB = bufs[(4 - k % 3) % 3];
            return f32 ? run_axis_only<float>(oo) : run_axis_only<double>(oo);
        };
        if ((err = run_on(0)) != hipSuccess) break;
        if ((err = hipEventRecord(e0, o.stream)) != hipSuccess) break;
        for (int r = 1; r <= 3 && err == hipSuccess; r++) err = run_on(r);
        if (err != hipSuccess || (err = hipEventRecord(e1, o.stream)) != hipSuccess) break;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.0f;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        tune_log("axis", f32, P, 0, ms);
        if (ms < best_ms) {
            best_ms = ms;
            best = P;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return FGH_E_DEVICE;
    op->P_axis = best;
    op->lds_axis = lds_of(best);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = best;
    return FGH_OK;
}

// Tile width of the middle pass, measured at plan creation.  The per-column arithmetic does not
// depend on the width (results are identical for every choice); the best width depends on how
// the tile count meets the resident workgroups of the CUs, so a few widths are timed once per
// process and shape and the fastest is kept.  FGH_TUNE=0 keeps the static choice.
fgh_status tune_middle(fgh_plan p, OpPlan* op, bool f32)
{
    if (!op->v2_mid || env_int("FGH_TUNE", 1) == 0 || env_int("FGH_P_EXACT", 0) != 0) return FGH_OK;
    static std::mutex mu;
    static std::map<std::vector<long long>, std::pair<int, int>> cache;
    const Geo& g = op->g;
    const std::vector<long long> key = {f32 ? 1 : 0, g.d, g.L[0], g.B[0], g.B[1], g.Hb, g.cols_mid};
    const size_t cs = f32 ? 8 : 16;
    auto lds_of = [&](int P, int pad) { return (size_t)(g.L[0] + (size_t)g.d * P * (g.L[0] + pad)) * cs; };
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            op->P_mid = it->second.first;
            op->mid_pad = it->second.second;
            op->lds_mid = lds_of(op->P_mid, op->mid_pad);
            return FGH_OK;
        }
    }
    // 7 is not tried: its 112-byte FP64 row segments split cache lines and add ~9 % written bytes
    const int cand[] = {4, 5, 6, 8, 9, 10, 12, 16};
    hipEvent_t e0, e1;
    HIPOK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FGH_E_DEVICE;
    }
    int best = op->P_mid, best_pad = 0;
    float best_ms = 1e30f;
    void* const bufs[3] = {g.d == 3 ? op->SB : op->SA, g.d == 3 ? op->SA : op->SB, p->ws + p->lay.vec64};
    hipError_t err = hipSuccess;
    for (int round = 0; round < 2 && err == hipSuccess; round++)
    for (int pad = 0; pad < 2 && err == hipSuccess; pad++)
        for (int P : cand) {
            if (lds_of(P, pad) > 128 * 1024 || P > g.cols_mid) continue;
            OpPlan o = *op;
            o.P_mid = P;
            o.mid_pad = pad;
            o.lds_mid = lds_of(P, pad);
            o.prof = nullptr;
            // the launches rotate over three buffers (the spectra and the vector storage, scratch
            // at this point): a pass repeated on one spectrum that fits the last-level cache would
            // be timed from the cache, not from HBM as in an application
            auto run_on = [&](int k) {
                OpPlan oo = o;
                (g.d == 3 ? oo.SB : oo.SA) = bufs[k % 3];
                return f32 ? run_middle_only<float>(oo) : run_middle_only<double>(oo);
            };
            if ((err = run_on(0)) != hipSuccess) break;
            if ((err = hipEventRecord(e0, o.stream)) != hipSuccess) break;
            for (int r = 1; r <= 3 && err == hipSuccess; r++) err = run_on(r);
            if (err != hipSuccess || (err = hipEventRecord(e1, o.stream)) != hipSuccess) break;
            if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.0f;
            if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            tune_log("middle", f32, P, pad, ms);
            if (ms < best_ms) {
                best_ms = ms;
                best = P;
                best_pad = pad;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return FGH_E_DEVICE;
    op->P_mid = best;
    op->mid_pad = best_pad;
    op->lds_mid = lds_of(best, best_pad);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = {best, best_pad};
    return FGH_OK;
}

// Rows per block of the specialised first pass, measured at plan creation like the middle pass's
// tile width.  Only even counts are tried: a tile then starts on an even real row, so rows are
// paired into complex transforms the same way whatever the choice, and results do not depend on
// it.
fgh_status tune_first(fgh_plan p, OpPlan* op, bool f32, const void* x)
{
    if (!op->v2_row || env_int("FGH_TUNE", 1) == 0 || std::getenv("FGH_RPB")) return FGH_OK;
    static std::mutex mu;
    static std::map<std::vector<long long>, int> cache;
    const Geo& g = op->g;
    // the timed pass is the identity-operator first pass: it does not read the coefficients
    const std::vector<long long> key = {f32 ? 1 : 0, g.d, g.L[g.d - 1], g.Hb, g.rows};
    const size_t cs = f32 ? 8 : 16;
    const size_t tabb = kMaxPhases * 6 * (f32 ? 4 : 8);
    const int L = g.L[g.d - 1];
    auto lds_of = [&](int r) { return (size_t)(L + (size_t)((r * g.d + 1) / 2) * L) * cs + tabb; };
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            op->rpb_first = it->second;
            op->lds_first_v2 = lds_of(it->second);
            return FGH_OK;
        }
    }
    const int cand[] = {6, 8, 10, 12, 16};
    hipEvent_t e0, e1;
    HIPOK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FGH_E_DEVICE;
    }
    int best = op->rpb_first;
    float best_ms = 1e30f;
    const void* const xs[3] = {x, f32 ? (const void*)p->p32 : (const void*)p->p64,
                               f32 ? (const void*)p->q32 : (const void*)p->q64};
    hipError_t err = hipSuccess;
    for (int round = 0; round < 2 && err == hipSuccess; round++)
    for (int r : cand) {
        if (lds_of(r) > 128 * 1024 || r > g.rows) continue;
        OpPlan o = *op;
        o.rpb_first = r;
        o.lds_first_v2 = lds_of(r);
        o.prof = nullptr;
        // launches cycle over three input vectors and two spectra (see tune_middle)
        auto run = [&](int k) {
            OpPlan oo = o;
            oo.SA = k & 1 ? op->SB : op->SA;
            return f32 ? run_first_only<float>(oo, static_cast<const float*>(xs[k % 3]))
                       : run_first_only<double>(oo, static_cast<const double*>(xs[k % 3]));
        };
        if ((err = run(0)) != hipSuccess) break;
        if ((err = hipEventRecord(e0, o.stream)) != hipSuccess) break;
        for (int k = 1; k <= 3 && err == hipSuccess; k++) err = run(k);
        if (err != hipSuccess || (err = hipEventRecord(e1, o.stream)) != hipSuccess) break;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.0f;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        tune_log("first", f32, r, 0, ms);
        if (ms < best_ms) {
            best_ms = ms;
            best = r;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return FGH_E_DEVICE;
    op->rpb_first = best;
    op->lds_first_v2 = lds_of(best);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = best;
    return FGH_OK;
}

// Whether CG defers its iterate update to the next body's first pass by default: when the loop's
// four vectors exceed the last-level cache (below it the update's x stream is served from the
// cache, and the first pass is faster with its own, larger chunks).
bool cg_defers(long long n, size_t bytes_per_real) { return 4.0 * (double)n * bytes_per_real > kLastLevelCacheBytes; }

// Rows per block of CG's first pass with the deferred iterate update (three vectors in, two out,
// per point), timed like the first pass's but with the operator itself: once the coefficients are
// set, on the plan's vectors as scratch, and only where CG defers the update by default.
fgh_status tune_first_cg(fgh_plan p, OpPlan* op, bool f32)
{
    if (!op->v2_row || env_int("FGH_TUNE", 1) == 0 || std::getenv("FGH_RPB")) return FGH_OK;
    const long long n = (long long)p->d * p->g.npts;
    if (!cg_defers(n, f32 ? 4 : 8)) return FGH_OK;
    static std::mutex mu;
    static std::map<std::vector<long long>, int> cache;
    const Geo& g = op->g;
    const std::vector<long long> key = {f32 ? 1 : 0, g.d, g.L[g.d - 1], g.Hb, g.rows, op->A.kind};
    const size_t cs = f32 ? 8 : 16;
    const size_t tabb = kMaxPhases * 6 * (f32 ? 4 : 8);
    const int L = g.L[g.d - 1];
    auto lds_of = [&](int r) { return (size_t)(L + (size_t)((r * g.d + 1) / 2) * L) * cs + tabb; };
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            op->rpb_first_x = it->second;
            op->lds_first_x = lds_of(it->second);
            return FGH_OK;
        }
    }
    // x, r, p: the plan's vectors (scratch until a solve), with defined values; alpha = beta = 0
    void* xs = f32 ? (void*)p->x32 : (void*)p->q64;
    void* rs = f32 ? (void*)p->r32 : (void*)p->r64;
    void* ps = f32 ? (void*)p->p32 : (void*)p->p64;
    if (f32) {
        HIPOK(run_fill<float>(p->stream, n, p->x32, 0.0f));
        HIPOK(run_fill<float>(p->stream, n, p->r32, 1.0f));
        HIPOK(run_fill<float>(p->stream, n, p->p32, 0.0f));
    } else {
        HIPOK(run_fill<double>(p->stream, n, p->q64, 0.0));
        HIPOK(run_fill<double>(p->stream, n, p->r64, 1.0));
        HIPOK(run_fill<double>(p->stream, n, p->p64, 0.0));
    }
    HIPOK(run_init_loop(*op, 0.0, 0.0, 0.0, -1.0, (double)g.npts, 0.0, 0.0, 0.0, 1));
    const int cand[] = {4, 6, 8, 10, 12, 16};
    hipEvent_t e0, e1;
    HIPOK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FGH_E_DEVICE;
    }
    int best = op->rpb_first_x;
    float best_ms = 1e30f;
    hipError_t err = hipSuccess;
    for (int round = 0; round < 2 && err == hipSuccess; round++)
    for (int r : cand) {
        if (lds_of(r) > 128 * 1024 || r > g.rows) continue;
        OpPlan o = *op;
        o.rpb_first_x = r;
        o.lds_first_x = lds_of(r);
        o.prof = nullptr;
        auto run = [&]() {
            return f32 ? run_first_cg_only<float>(o, static_cast<float*>(xs), static_cast<const float*>(rs),
                                                  static_cast<float*>(ps))
                       : run_first_cg_only<double>(o, static_cast<double*>(xs), static_cast<const double*>(rs),
                                                   static_cast<double*>(ps));
        };
        if ((err = run()) != hipSuccess) break;
        if ((err = hipEventRecord(e0, o.stream)) != hipSuccess) break;
        for (int k = 0; k < 3 && err == hipSuccess; k++) err = run();
        if (err != hipSuccess || (err = hipEventRecord(e1, o.stream)) != hipSuccess) break;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.0f;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        tune_log("first_cg", f32, r, 0, ms);
        if (ms < best_ms) {
            best_ms = ms;
            best = r;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return FGH_E_DEVICE;
    op->rpb_first_x = best;
    op->lds_first_x = lds_of(best);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = best;
    return FGH_OK;
}

// Rows per block of the fused last + first pass, measured at plan creation like the first pass's:
// the last pass's count and even counts above it (so the partial sums fit the buffer sized for
// the last pass, and rows pair into complex transforms as in the separate passes: results do not
// depend on the choice).
fgh_status tune_fused(fgh_plan p, OpPlan* op, bool f32, void* x)
{
    if (!op->v2_row || env_int("FGH_TUNE", 1) == 0 || std::getenv("FGH_RPB")) return FGH_OK;
    static std::mutex mu;
    static std::map<std::vector<long long>, int> cache;
    const Geo& g = op->g;
    const std::vector<long long> key = {f32 ? 1 : 0, g.d, g.L[g.d - 1], g.Hb, g.rows, (long long)op->A.kind,
                                        op->rpb};
    const size_t cs = f32 ? 8 : 16;
    const size_t tabb = kMaxPhases * 6 * (f32 ? 4 : 8);
    const int L = g.L[g.d - 1];
    auto lds_of = [&](int r) { return (size_t)(L + (size_t)((r * g.d + 1) / 2) * (L + 1)) * cs + 2 * tabb; };
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            op->rpb_fused = it->second;
            op->lds_fused = lds_of(it->second);
            return FGH_OK;
        }
    }
    std::vector<int> cand = {op->rpb};
    for (int r : {8, 10, 12, 16})
        if (r > op->rpb) cand.push_back(r);
    hipEvent_t e0, e1;
    HIPOK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return FGH_E_DEVICE;
    }
    int best = op->rpb_fused;
    float best_ms = 1e30f;
    hipError_t err = hipSuccess;
    for (int round = 0; round < 2 && err == hipSuccess; round++)
    for (int r : cand) {
        if (lds_of(r) > 128 * 1024 || r > g.rows) continue;
        OpPlan o = *op;
        o.rpb_fused = r;
        o.lds_fused = lds_of(r);
        auto run = [&]() {
            return f32 ? run_fused_only<float>(o, static_cast<float*>(x)) : run_fused_only<double>(o, static_cast<double*>(x));
        };
        if ((err = run()) != hipSuccess) break;
        if ((err = hipEventRecord(e0, o.stream)) != hipSuccess) break;
        for (int k = 0; k < 3 && err == hipSuccess; k++) err = run();
        if (err != hipSuccess || (err = hipEventRecord(e1, o.stream)) != hipSuccess) break;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.0f;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        tune_log("fused", f32, r, 0, ms);
        if (ms < best_ms) {
            best_ms = ms;
            best = r;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return FGH_E_DEVICE;
    op->rpb_fused = best;
    op->lds_fused = lds_of(best);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = best;
    return FGH_OK;
}

// Read one device double (synchronises the stream).
fgh_status read_scalar(fgh_plan p, const double* dev, double* out)
{
    HIPOK(hipMemcpyAsync(p->host_buf, dev, sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIPOK(hipStreamSynchronize(p->stream));
    *out = p->host_buf[0];
    return FGH_OK;
}

fgh_status reduce_read(fgh_plan p, const OpPlan& op, int n, int redop, double* out)
{
    HIPOK(run_reduce_async(op, n, redop));
    return read_scalar(p, &op.sc->total, out);
}

template <typename T>
const OpPlan& opp(fgh_plan p);
template <>
const OpPlan& opp<double>(fgh_plan p) { return p->op64; }
template <>
const OpPlan& opp<float>(fgh_plan p) { return p->op32; }

// ||b||^2 (raw sum) of b = -G A E into r; also ||A E||^2.
template <typename T>
fgh_status rhs(fgh_plan p, const double* E, T* r, double* bb, double* ae2)
{
    const OpPlan& op = opp<T>(p);
    ApplyArgs a;
    a.op = OP_E;
    a.epi = EPI_STORE;
    a.sgn = -1.0;
    for (int c = 0; c < p->d; c++) a.E[c] = E[c];
    a.y = r;
    int nb = 0;
    HIPOK(run_apply<T>(op, a, &nb));
    fgh_status st = reduce_read(p, op, nb, RED_SET_RR, bb);
    if (st) return st;
    if (ae2) {
        HIPOK(run_norm_AE(p->op64, E, &nb));
        double v;
        st = reduce_read(p, p->op64, nb, RED_TOTAL, &v);
        if (st) return st;
        *ae2 = v;
    }
    return FGH_OK;
}

struct SolveOut {
    int iters = 0;
    int status = FGH_OK;
    double res = 0.0;   // stopping-test quantity at exit, relative to its scale
};

static_assert(sizeof(Scalars) <= 64 * sizeof(double), "pinned readback buffer too small");

constexpr int kGraphBodies = 8;

uint64_t mix_key(uint64_t h, uint64_t v)
{
    h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    return h;
}
uint64_t key_of(std::initializer_list<uint64_t> vals)
{
    uint64_t h = 1469598103934665603ULL;
    for (uint64_t v : vals) h = mix_key(h, v);
    return h;
}
uint64_t bits(double v)
{
    uint64_t u;
    std::memcpy(&u, &v, sizeof u);
    return u;
}
uint64_t bits(const void* ptr) { return (uint64_t)(uintptr_t)ptr; }

bool graphs_enabled()
{
    const char* v = std::getenv("FGH_GRAPHS");
    return !(v && v[0] == '0');
}

void drop_graph(fgh_plan p)
{
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->gexec = nullptr;
    p->graph = nullptr;
    p->gkey = 0;
}

// Run loop bodies in chunks; the device decides when to stop (Scalars::done) and counts the
// bodies, so the host synchronises once per chunk instead of once per body.  When the plan's
// stream can be captured, kGraphBodies bodies are captured once into a HIP graph (keyed by the
// body's operands) and the graph is replayed; otherwise the bodies are launched one by one.
template <typename Body>
fgh_status run_loop(fgh_plan p, const OpPlan& op, Body body, uint64_t key, bool fixed, double scale, SolveOut* out)
{
    const Scalars* h = reinterpret_cast<const Scalars*>(p->host_buf);
    const bool use_graph = graphs_enabled() && !op.prof && op.stream != nullptr;
    if (p->hist_fn) {
        // history scale of the stopping-test quantity and its value before the first body
        const double hv[2] = {scale > 0 ? 1.0 / scale : 1.0, 1.0};
        HIPOK(hipMemcpyAsync(op.sc->aux + 12, hv, sizeof hv, hipMemcpyHostToDevice, op.stream));
        HIPOK(p->hist_fn());
        key = mix_key(key, p->hist_key);
    }
    auto step = [&]() -> hipError_t {
        hipError_t e = body();
        if (e != hipSuccess || !p->hist_fn) return e;
        return p->hist_fn();
    };
    if (use_graph && (p->gkey != key || !p->gexec)) {
        drop_graph(p);
        HIPOK(hipStreamBeginCapture(op.stream, hipStreamCaptureModeThreadLocal));
        hipError_t ce = hipSuccess;
        for (int k = 0; k < kGraphBodies && ce == hipSuccess; k++) ce = step();
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(op.stream, &g);
        if (ce != hipSuccess || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return FGH_E_DEVICE;
        }
        p->graph = g;
        HIPOK(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
        p->gkey = key;
    }
    int chunk = 1;
    for (;;) {
        for (int k = 0; k < chunk; k++) {
            if (use_graph) {
                HIPOK(hipGraphLaunch(p->gexec, op.stream));
            } else {
                for (int b = 0; b < kGraphBodies; b++) HIPOK(step());
            }
        }
        HIPOK(hipMemcpyAsync(p->host_buf, op.sc, sizeof(Scalars), hipMemcpyDeviceToHost, op.stream));
        HIPOK(hipStreamSynchronize(op.stream));
        if (h->done) break;
        if (chunk < 4) chunk *= 2;
    }
    out->iters = h->m;
    out->res = scale > 0 ? h->last / scale : h->last;
    if (h->done == 3)
        out->status = FGH_E_DIVERGED;
    else if (h->done == 2 && !fixed)
        out->status = FGH_E_NO_CONVERGENCE;
    else
        out->status = FGH_OK;
    return FGH_OK;
}

// One body of Algorithm 2: p <- r + beta p (beta = 0 before the first body, p = r), q = C p,
// alpha = (r, r) / (q, p), x += alpha p, r -= alpha q, beta = (r_new, r_new) / (r, r).  The
// coefficients are left in the loop's scalar block.  With defer_x the body's x += alpha p is left
// to the next body's first pass, which reads p there anyway before replacing it (one vector
// stream less per body; the same operation on the same values), and the loop's last update to
// run_cg_x after the loop.
template <typename T>
hipError_t cg_body(const OpPlan& op, long long n, T* x, T* r, T* pv, T* q, bool defer_x)
{
    ApplyArgs a;
    a.op = OP_AP_CG;
    a.p_cg = pv;
    a.r_cg = r;
    a.x_cg = defer_x ? x : nullptr;
    a.epi = EPI_CG;
    a.eq = q;
    a.ep = pv;
    a.loop = true;
    int nb = 0;
    hipError_t e = run_apply<T>(op, a, &nb);
    if (e != hipSuccess) return e;
    if ((e = run_reduce_async(op, nb, RED_CG_ALPHA)) != hipSuccess) return e;
    if ((e = run_cg_update<T>(op, n, defer_x ? nullptr : x, r, pv, q)) != hipSuccess) return e;
    return run_reduce_async(op, vec_blocks(), RED_CG_END);
}

// Conjugate gradients (Algorithm 2) for C x = b with b already in r, x = 0 on entry.  Stops when
// ||r_m|| <= tol_rel ||b|| (recursive residual) or after `fixed` bodies.  The iterate update is
// deferred to the next body (cg_body) on large grids unless a history recorder reads x between
// bodies.
template <typename T>
fgh_status cg_core(fgh_plan p, T* x, T* r, T* pv, T* q, double tol_rel, int max_iter, int fixed, SolveOut* out)
{
    const OpPlan& op = opp<T>(p);
    const long long n = (long long)p->d * p->g.npts;
    const double S = (double)p->g.npts;
    HIPOK(run_copy<T>(p->stream, n, pv, r));
    double bb = 0.0;
    {
        int nb = 0;
        HIPOK(run_dot<T>(op, n, r, r, &nb));
        fgh_status st0 = reduce_read(p, op, nb, RED_TOTAL, &bb);
        if (st0) return st0;
    }
    const double normb = std::sqrt(bb / S);
    const int limit = fixed > 0 ? fixed : max_iter;
    // alpha = 0 before the first body: its deferred update leaves x as it is
    HIPOK(run_init_loop(op, bb, 0.0, 0.0, fixed > 0 ? -1.0 : tol_rel * normb, S, 0.0, 0.0, 0.0, limit));
    // deferral saves the update's x stream from HBM, on grids where it reaches HBM (cg_defers;
    // FGH_CG_DEFER=1 or 0 forces it on or off)
    const int force = env_int_any("FGH_CG_DEFER", -1);
    const bool defer_x = !p->hist_fn && (force >= 0 ? force == 1 : cg_defers(n, sizeof(T)));
    auto body = [&]() { return cg_body<T>(op, n, x, r, pv, q, defer_x); };
    const uint64_t key = key_of({defer_x ? 2u : 1u, sizeof(T), bits(x), bits(r), bits(pv), bits(q)});
    const fgh_status s = run_loop(p, op, body, key, fixed > 0, normb, out);
    // the last body's x += alpha p (bodies after the stop return at once and leave alpha and p)
    if (s == FGH_OK && defer_x) HIPOK(run_cg_x<T>(op, n, x, pv));
    return s;
}

// Fused loop bodies (the last pass also runs the next body's first pass; the loop's first body
// gets its first pass from a prologue): with the specialised row kernels, and not while a history
// recorder is armed (its monitors may apply operators on the plan's spectrum buffers between
// bodies).  FGH_FUSE=0 turns fusion off.
bool fuse_loop(fgh_plan p, const OpPlan& op)
{
    const char* v = std::getenv("FGH_FUSE");
    return fusable(op) && !p->hist_fn && !(v && v[0] == '0');
}

// Deferred loop reductions (see ApplyArgs::defer_redop): with fused bodies in 3D with the
// specialised axis kernels.  The host then sees a body's stopping test one body later, so a loop
// may launch one more chunk of bodies that return at once.  FGH_DEFER=0 turns this off.
bool defer_reduction(const OpPlan& op, bool fuse)
{
    const char* v = std::getenv("FGH_DEFER");
    return fuse && op.g.d == 3 && op.v2_axis && op.v2_row && !(v && v[0] == '0');
}

// The loop's prologue of a fused loop: the first body's first pass alone.
template <typename T>
hipError_t fused_prologue(const OpPlan& op, ApplyArgs a)
{
    a.first_only = true;
    a.loop = false;
    int nb = 0;
    return run_apply<T>(op, a, &nb);
}

// Chebyshev semi-iteration (Algorithm 3), b in r, x = 0, on the interval [delta - c, delta + c]
// (c < 0: the plan's [c_A, C_A]).  With c = 0 the coefficients stay alpha = 1/delta, beta = 0:
// that is Richardson's iteration x += (1/delta)(b - C x) on an explicit right-hand side.
template <typename T>
fgh_status cheb_core(fgh_plan p, T* x, T* r, T* pv, double tol_rel, int max_iter, int fixed, SolveOut* out,
                     double c_in = -1.0, double delta_in = 0.0)
{
    const OpPlan& op = opp<T>(p);
    const long long n = (long long)p->d * p->g.npts;
    const double S = (double)p->g.npts;
    HIPOK(run_copy<T>(p->stream, n, pv, r));
    double bb = 0.0;
    {
        int nb = 0;
        HIPOK(run_dot<T>(op, n, r, r, &nb));
        fgh_status st0 = reduce_read(p, op, nb, RED_TOTAL, &bb);
        if (st0) return st0;
    }
    const double normb = std::sqrt(bb / S);
    const double c = c_in >= 0.0 ? c_in : 0.5 * (p->CA - p->cA);
    const double delta = c_in >= 0.0 ? delta_in : 0.5 * (p->cA + p->CA);
    const int limit = fixed > 0 ? fixed : max_iter;
    HIPOK(run_init_loop(op, bb, 1.0 / delta, -0.5 * (c / delta) * (c / delta), fixed > 0 ? -1.0 : tol_rel * normb, S,
                        0.0, c, delta, limit));
    const bool fuse = fuse_loop(p, op);
    ApplyArgs a;
    a.op = OP_AX;
    a.x = pv;
    a.epi = EPI_CHEB;
    a.ex = x;
    a.er = r;
    a.ep = pv;
    a.loop = true;
    a.cheb_dev = true;
    if (fuse) {
        HIPOK(fused_prologue<T>(op, a));
        a.skip_first = true;
        a.next_op = OP_AX;
    }
    const bool defer = defer_reduction(op, fuse);
    a.defer_redop = defer ? RED_CHEB_END : -1;
    auto body = [&]() -> hipError_t {
        int nb = 0;
        hipError_t e = run_apply<T>(op, a, &nb);
        if (e != hipSuccess || defer) return e;
        return run_reduce_async(op, nb, RED_CHEB_END);
    };
    const uint64_t key = key_of({2, sizeof(T), bits(x), bits(r), bits(pv), (uint64_t)fuse, (uint64_t)defer, bits(c),
                                 bits(delta)});
    return run_loop(p, op, body, key, fixed > 0, normb, out);
}

// Richardson (Algorithm 1): step = -w G A (E0 + x); stops when ||x_m - x_{m-1}|| <= thr.
template <typename T>
fgh_status rich_core(fgh_plan p, T* x, const double* E0, double thr, int max_iter, int fixed, double scale,
                     SolveOut* out)
{
    const OpPlan& op = opp<T>(p);
    const double S = (double)p->g.npts;
    const double omega = 2.0 / (p->cA + p->CA);
    const int limit = fixed > 0 ? fixed : max_iter;
    HIPOK(run_init_loop(op, 0.0, 0.0, 0.0, fixed > 0 ? -1.0 : thr, S, 0.0, 0.0, 0.0, limit));
    const bool fuse = fuse_loop(p, op);
    ApplyArgs a;
    a.op = OP_AX;
    a.x = x;
    for (int c = 0; c < p->d; c++) a.E[c] = E0[c];
    a.epi = EPI_RICH;
    a.ex = x;
    a.omega = omega;
    a.loop = true;
    if (fuse) {
        HIPOK(fused_prologue<T>(op, a));
        a.skip_first = true;
        a.next_op = OP_AX;
    }
    const bool defer = defer_reduction(op, fuse);
    a.defer_redop = defer ? RED_STEP_END : -1;
    auto body = [&]() -> hipError_t {
        int nb = 0;
        hipError_t e = run_apply<T>(op, a, &nb);
        if (e != hipSuccess || defer) return e;
        return run_reduce_async(op, nb, RED_STEP_END);
    };
    const uint64_t key = key_of({3, sizeof(T), bits(x), bits(E0[0]), bits(E0[1]), bits(p->d == 3 ? E0[2] : 0.0),
                                 bits(omega), (uint64_t)fuse, (uint64_t)defer});
    return run_loop(p, op, body, key, fixed > 0, scale, out);
}

// Eyre-Milton (Algorithm 4).  Plain form (src == NULL): x holds E + e; correction form
// (src != NULL): x holds delta, the source field is the double-precision defect.
template <typename T>
fgh_status em_core(fgh_plan p, T* x, const double* E, const T* src, double thr, int max_iter, int fixed,
                   double scale, SolveOut* out)
{
    const OpPlan& op = opp<T>(p);
    const double S = (double)p->g.npts;
    const double omega = std::sqrt(p->cA * p->CA);
    const int limit = fixed > 0 ? fixed : max_iter;
    HIPOK(run_init_loop(op, 0.0, 0.0, 0.0, fixed > 0 ? -1.0 : thr, S, 1e12 * (scale > 0 ? scale : 1.0), 0.0, 0.0,
                        limit));
    const bool fuse = fuse_loop(p, op);
    ApplyArgs a;
    a.op = OP_EM;
    a.x = x;
    a.omega = omega;
    a.mult = MULT_EM;
    a.epi = EPI_EM;
    a.ex = x;
    a.src = src;
    for (int c = 0; c < p->d; c++) a.E[c] = E[c];
    a.loop = true;
    if (fuse) {
        HIPOK(fused_prologue<T>(op, a));
        a.skip_first = true;
        a.next_op = OP_EM;
    }
    const bool defer = defer_reduction(op, fuse);
    a.defer_redop = defer ? RED_STEP_END : -1;
    auto body = [&]() -> hipError_t {
        int nb = 0;
        hipError_t e = run_apply<T>(op, a, &nb);
        if (e != hipSuccess || defer) return e;
        return run_reduce_async(op, nb, RED_STEP_END);
    };
    const uint64_t key = key_of({4, sizeof(T), bits(x), bits(src), bits(E[0]), bits(E[1]),
                                 bits(p->d == 3 ? E[2] : 0.0), bits(omega), (uint64_t)fuse, (uint64_t)defer});
    return run_loop(p, op, body, key, fixed > 0, scale, out);
}

// ||b - C e|| / ||b|| for the fluctuation e (double): apply C to (E + e) and compare with 0.
fgh_status true_residual(fgh_plan p, const double* E, const double* e, double bb, double* out)
{
    ApplyArgs a;
    a.op = OP_AX;
    a.x = e;
    for (int c = 0; c < p->d; c++) a.E[c] = E[c];
    a.epi = EPI_STORE;
    a.sgn = 1.0;
    a.y = p->q64;
    int nb = 0;
    HIPOK(run_apply<double>(p->op64, a, &nb));
    double v;
    fgh_status st = reduce_read(p, p->op64, nb, RED_TOTAL, &v);
    if (st) return st;
    *out = bb > 0 ? std::sqrt(v / bb) : std::sqrt(v / (double)p->g.npts);
    return FGH_OK;
}

// History entry of plan p's loop for the iterate x (device [d][grid]) at the current body count.
// Plain: the energy (A(E + x), E + x) on the integration grid, with E read from the loop's
// scalar block (aux[0..3), or the zeros at aux[3..6) when x is the whole field of Eyre-Milton).
// Bound monitor (GaNi plan with a Ga plan): the energy of E + R G_N x on the double grid, the
// guaranteed bound of the iterate (eq:guar_upper_bound_m); G_N also strips the mean of a whole
// field, so E is added in either case.
hipError_t hist_record(fgh_plan p, const double* x, bool whole)
{
    const OpPlan& op = p->op64;
    const int nvals = 1 + p->d;
    hipError_t e;
    if ((p->hist_nc || p->hist_mean) &&
        (e = run_hist_nonconf(op, x, op.sc->aux + (whole ? 0 : 3), p->hist_scratch, p->hist_nc, p->hist_mean,
                              p->hist_cap)) != hipSuccess)
        return e;
    if (!p->hist_en) return run_hist(op.stream, op.partials, 0, nvals, op.sc, p->hist_res, nullptr, p->hist_cap, 0.0);
    int nb = 0;
    if (!p->hist_ga) {
        if ((e = run_effective(op, 1, op.sc->aux + (whole ? 3 : 0), x, &nb)) != hipSuccess) return e;
        return run_hist(op.stream, op.partials, nb, nvals, op.sc, p->hist_res, p->hist_en, p->hist_cap,
                        1.0 / (double)p->g.npts);
    }
    fgh_plan ga = p->hist_ga;
    OpPlan opn = op;
    opn.prof = nullptr;
    OpPlan opm = ga->op64;
    opm.stream = op.stream;
    opm.prof = nullptr;
    ApplyArgs a;  // ga->r64 <- G_N x
    a.op = OP_ID;
    a.x = x;
    a.mult = MULT_G;
    a.epi = EPI_STORE;
    a.sgn = 1.0;
    a.y = ga->r64;
    if ((e = run_apply<double>(opn, a, &nb)) != hipSuccess) return e;
    if ((e = run_prolong(opn, opm, ga->r64, ga->q64)) != hipSuccess) return e;
    if ((e = run_effective(opm, 1, opm.sc->aux, ga->q64, &nb)) != hipSuccess) return e;
    return run_hist(op.stream, opm.partials, nb, nvals, op.sc, p->hist_res, p->hist_en, p->hist_cap,
                    1.0 / (double)ga->g.npts);
}

// Arms the history recorder for load j of a solve (x: the loop's iterate).
fgh_status hist_arm(fgh_plan p, const double* E, int j, const double* x, bool whole)
{
    if (!p->hist_res && !p->hist_en && !p->hist_nc && !p->hist_mean) return FGH_OK;
    double v[15] = {0};
    for (int c = 0; c < p->d; c++) v[c] = E[c];
    v[14] = (double)((long long)j * p->hist_cap);
    HIPOK(hipMemcpyAsync(p->op64.sc->aux, v, sizeof v, hipMemcpyHostToDevice, p->stream));
    if (p->hist_ga) HIPOK(hipMemcpyAsync(p->hist_ga->op64.sc->aux, v, 3 * sizeof(double), hipMemcpyHostToDevice,
                                         p->stream));
    p->hist_fn = [p, x, whole]() { return hist_record(p, x, whole); };
    p->hist_key = key_of({7, bits(p->hist_res), bits(p->hist_en), bits(p->hist_nc), bits(p->hist_mean),
                          bits(p->hist_scratch), (uint64_t)p->hist_cap, bits(p->hist_ga), bits(x), (uint64_t)whole});
    return FGH_OK;
}

fgh_status solve_one_fp64(fgh_plan p, int solver, const double* E, double tol, int max_iter, int fixed, double* e,
                          fgh_stats* st, int load)
{
    struct Disarm {
        fgh_plan p;
        ~Disarm() { p->hist_fn = nullptr; }
    } disarm{p};
    const long long n = (long long)p->d * p->g.npts;
    const double S = (double)p->g.npts;
    double normE = 0.0;
    for (int c = 0; c < p->d; c++) normE += E[c] * E[c];
    normE = std::sqrt(normE);
    SolveOut so;
    double bb = 0.0, ae2 = 0.0;
    fgh_status s;
    if (solver == FGH_CG || solver == FGH_CHEBYSHEV) {
        if ((s = rhs<double>(p, E, p->r64, &bb, &ae2))) return s;
        HIPOK(run_fill<double>(p->stream, n, e, 0.0));
        const bool zero = !(std::sqrt(bb / S) > kZeroRhs * std::sqrt(ae2 / S));
        if ((s = hist_arm(p, E, load, e, false))) return s;
        if (zero) {
            so.iters = 0;
            so.res = 0.0;
            if (p->hist_fn) {  // the single entry m = 0 with the test quantity 0
                HIPOK(run_init_loop(p->op64, 0.0, 0.0, 0.0, -1.0, S, 0.0, 0.0, 0.0, 0));
                const double hv[2] = {1.0, 0.0};
                HIPOK(hipMemcpyAsync(p->op64.sc->aux + 12, hv, sizeof hv, hipMemcpyHostToDevice, p->stream));
                HIPOK(p->hist_fn());
            }
        } else if (solver == FGH_CG) {
            if ((s = cg_core<double>(p, e, p->r64, p->p64, p->q64, tol, max_iter, fixed, &so))) return s;
        } else {
            if ((s = cheb_core<double>(p, e, p->r64, p->p64, tol, max_iter, fixed, &so))) return s;
        }
    } else if (solver == FGH_RICHARDSON) {
        HIPOK(run_fill<double>(p->stream, n, e, 0.0));
        if ((s = hist_arm(p, E, load, e, false))) return s;
        if ((s = rich_core<double>(p, e, E, tol * normE, max_iter, fixed, normE, &so))) return s;
    } else {
        HIPOK(run_fill_field<double>(p->stream, p->d, p->g.npts, e, E));
        if ((s = hist_arm(p, E, load, e, true))) return s;
        if ((s = em_core<double>(p, e, E, nullptr, tol * normE, max_iter, fixed, normE, &so))) return s;
        double negE[3] = {-E[0], -E[1], p->d == 3 ? -E[2] : 0.0};
        // e <- x - E
        HIPOK(run_fill_field<double>(p->stream, p->d, p->g.npts, p->q64, negE));
        HIPOK(run_add_f64(p->stream, n, e, p->q64));
    }
    if (st) {
        st->iters = so.iters;
        st->outer_iters = 0;
        st->fp64_applies = so.iters;
        st->status = so.status;
        st->rel_res_recursive = so.res;
    }
    return FGH_OK;
}

// Defect correction: FP64 outer loop, FP32 inner solves (the same algorithm as `solver`).
//  CG / Chebyshev: r = b - C x in FP64, inner FP32 solve of C delta = r to the relative
//    tolerance max(tol ||b|| / ||r||, kInnerTolMin), then x += G delta in FP64 (the projection
//    removes the FP32 round-off that is not curl-free, so the iterate stays conforming);
//    stop when ||b - C x|| <= tol ||b||.
//  Richardson: stop when the next FP64 step w ||b - C x|| is <= tol |E| (and take it); the
//    correction solves C delta = r by Richardson in FP32 to the relative residual
//    max(tol |E| / (w ||r||), kInnerTolMin), then x += G delta in FP64.
//  Eyre-Milton: the FP64 defect dbar = EM(x) - x; the correction delta obeys
//    delta = (A + wI)^{-1} (I - 2G^)(A - wI) delta + dbar (same contraction as Algorithm 4),
//    iterated in FP32 from delta = 0; x += delta; stop when ||dbar|| <= tol |E| (then x takes
//    that last FP64 step, as Algorithm 4 would).
fgh_status solve_one_refined(fgh_plan p, int solver, const double* E, double tol, int max_iter, double* e,
                             fgh_stats* st)
{
    const long long n = (long long)p->d * p->g.npts;
    const double S = (double)p->g.npts;
    double normE = 0.0;
    for (int c = 0; c < p->d; c++) normE += E[c] * E[c];
    normE = std::sqrt(normE);
    int inner_total = 0, outer = 0, applies64 = 0, status = FGH_OK;
    double res = 0.0;
    fgh_status s;
    if (solver == FGH_EYRE_MILTON) {
        const double omega = std::sqrt(p->cA * p->CA);
        HIPOK(run_fill_field<double>(p->stream, p->d, p->g.npts, e, E));  // x = E
        bool done = false;
        for (outer = 0; outer < 200 && !done; outer++) {
            // r64 = EM(x) in FP64; the epilogue sums |EM(x) - x|^2
            HIPOK(run_copy<double>(p->stream, n, p->r64, e));
            ApplyArgs a;
            a.op = OP_EM;
            a.x = p->r64;
            a.omega = omega;
            a.mult = MULT_EM;
            a.epi = EPI_EM;
            a.ex = p->r64;
            for (int c = 0; c < p->d; c++) a.E[c] = E[c];
            int nb = 0;
            HIPOK(run_apply<double>(p->op64, a, &nb));
            applies64++;
            double dd;
            if ((s = reduce_read(p, p->op64, nb, RED_TOTAL, &dd))) return s;
            const double dnorm = std::sqrt(dd / S);
            res = normE > 0 ? dnorm / normE : dnorm;
            if (!std::isfinite(dnorm) || dnorm > 1e12 * (normE > 0 ? normE : 1.0)) {
                status = FGH_E_DIVERGED;
                break;
            }
            if (dnorm <= tol * normE) {
                HIPOK(run_copy<double>(p->stream, n, e, p->r64));
                done = true;
                break;
            }
            // dbar = EM(x) - x  (q64), its FP32 copy is the inner source
            HIPOK(run_axpby(p->stream, n, p->q64, 1.0, p->r64, 0.0));
            HIPOK(run_axpby(p->stream, n, p->q64, -1.0, e, 1.0));
            HIPOK(run_f64_to_f32(p->stream, n, p->r32, p->q64));
            HIPOK(run_fill<float>(p->stream, n, p->x32, 0.0f));
            double eta = tol * normE / dnorm;
            if (eta < kInnerTolMin) eta = kInnerTolMin;
            SolveOut so;
            if ((s = em_core<float>(p, p->x32, E, p->r32, eta * dnorm, max_iter, 0, dnorm, &so))) return s;
            inner_total += so.iters;
            if (so.status == FGH_E_DIVERGED) {
                status = FGH_E_DIVERGED;
                break;
            }
            HIPOK(run_add_f32_to_f64(p->stream, n, e, p->x32));
        }
        if (status == FGH_OK && !done) status = FGH_E_NO_CONVERGENCE;
        // fluctuation e = x - E
        double negE[3] = {-E[0], -E[1], p->d == 3 ? -E[2] : 0.0};
        HIPOK(run_fill_field<double>(p->stream, p->d, p->g.npts, p->q64, negE));
        HIPOK(run_add_f64(p->stream, n, e, p->q64));
    } else if (solver == FGH_CG || solver == FGH_CHEBYSHEV) {
        HIPOK(run_fill<double>(p->stream, n, e, 0.0));
        double bb = 0.0, ae2 = 0.0;
        if ((s = rhs<double>(p, E, p->r64, &bb, &ae2))) return s;
        applies64++;
        const bool zero = !(std::sqrt(bb / S) > kZeroRhs * std::sqrt(ae2 / S));
        const double normb = std::sqrt(bb / S);
        double rr = bb;
        if (!zero) {
            for (outer = 0; outer < 64; outer++) {
                if (outer > 0) {
                    // r = b - C x = -G A (E + x)
                    ApplyArgs a;
                    a.op = OP_AX;
                    a.x = e;
                    for (int c = 0; c < p->d; c++) a.E[c] = E[c];
                    a.epi = EPI_STORE;
                    a.sgn = -1.0;
                    a.y = p->r64;
                    int nb = 0;
                    HIPOK(run_apply<double>(p->op64, a, &nb));
                    applies64++;
                    if ((s = reduce_read(p, p->op64, nb, RED_TOTAL, &rr))) return s;
                }
                res = std::sqrt(rr / S) / normb;
                if (!std::isfinite(rr)) {
                    status = FGH_E_DIVERGED;
                    break;
                }
                if (res <= tol) break;
                double eta = tol / res;
                if (eta < kInnerTolMin) eta = kInnerTolMin;
                HIPOK(run_f64_to_f32(p->stream, n, p->r32, p->r64));
                HIPOK(run_fill<float>(p->stream, n, p->x32, 0.0f));
                SolveOut so;
                if (solver == FGH_CG) {
                    if ((s = cg_core<float>(p, p->x32, p->r32, p->p32, p->q32, eta, max_iter, 0, &so))) return s;
                } else {
                    if ((s = cheb_core<float>(p, p->x32, p->r32, p->p32, eta, max_iter, 0, &so))) return s;
                }
                inner_total += so.iters;
                if (so.status == FGH_E_DIVERGED) {
                    status = FGH_E_DIVERGED;
                    break;
                }
                // x += G delta in FP64
                HIPOK(run_fill<double>(p->stream, n, p->p64, 0.0));
                HIPOK(run_add_f32_to_f64(p->stream, n, p->p64, p->x32));
                ApplyArgs a;
                a.op = OP_ID;
                a.x = p->p64;
                a.epi = EPI_STORE;
                a.sgn = 1.0;
                a.y = p->q64;
                int nb = 0;
                HIPOK(run_apply<double>(p->op64, a, &nb));
                applies64++;
                HIPOK(run_add_f64(p->stream, n, e, p->q64));
            }
            if (status == FGH_OK && !(res <= tol)) status = FGH_E_NO_CONVERGENCE;
        }
    } else if (solver == FGH_RICHARDSON) {
        // Algorithm 1's step from an iterate x is w (b - C x), so its stopping test on the step norm
        // is a test on the FP64 residual: stop once w ||b - C x|| <= tol |E|, after taking that
        // last step.  Until then the correction solves C delta = r by Richardson's iteration in
        // FP32 (Chebyshev on the one-point interval [delta, delta], delta = 1/w, is exactly that
        // iteration on an explicit right-hand side): its step norms are w times its residuals, so
        // it stops on ||r_k|| <= eta ||r||.
        const double omega = 2.0 / (p->cA + p->CA);
        HIPOK(run_fill<double>(p->stream, n, e, 0.0));
        double bb = 0.0;
        if ((s = rhs<double>(p, E, p->r64, &bb, nullptr))) return s;
        applies64++;
        double rr = bb;
        bool done = false;
        for (outer = 0; outer < 64; outer++) {
            if (outer > 0) {
                // r = b - C x = -G A (E + x)
                ApplyArgs a;
                a.op = OP_AX;
                a.x = e;
                for (int c = 0; c < p->d; c++) a.E[c] = E[c];
                a.epi = EPI_STORE;
                a.sgn = -1.0;
                a.y = p->r64;
                int nb = 0;
                HIPOK(run_apply<double>(p->op64, a, &nb));
                applies64++;
                if ((s = reduce_read(p, p->op64, nb, RED_TOTAL, &rr))) return s;
            }
            const double step = omega * std::sqrt(rr / S);
            res = normE > 0 ? step / normE : step;
            if (!std::isfinite(rr)) {
                status = FGH_E_DIVERGED;
                break;
            }
            if (step <= tol * normE) {
                HIPOK(run_axpby(p->stream, n, e, omega, p->r64, 1.0));  // the last step, x += w r
                done = true;
                break;
            }
            double eta = tol * normE / step;
            if (eta < kInnerTolMin) eta = kInnerTolMin;
            HIPOK(run_f64_to_f32(p->stream, n, p->r32, p->r64));
            HIPOK(run_fill<float>(p->stream, n, p->x32, 0.0f));
            SolveOut so;
            if ((s = cheb_core<float>(p, p->x32, p->r32, p->p32, eta, max_iter, 0, &so, 0.0, 1.0 / omega))) return s;
            inner_total += so.iters;
            if (so.status == FGH_E_DIVERGED) {
                status = FGH_E_DIVERGED;
                break;
            }
            // x += G delta in FP64
            HIPOK(run_fill<double>(p->stream, n, p->p64, 0.0));
            HIPOK(run_add_f32_to_f64(p->stream, n, p->p64, p->x32));
            ApplyArgs a;
            a.op = OP_ID;
            a.x = p->p64;
            a.epi = EPI_STORE;
            a.sgn = 1.0;
            a.y = p->q64;
            int nb = 0;
            HIPOK(run_apply<double>(p->op64, a, &nb));
            applies64++;
            HIPOK(run_add_f64(p->stream, n, e, p->q64));
        }
        if (status == FGH_OK && !done) status = FGH_E_NO_CONVERGENCE;
    } else {
        return FGH_E_UNSUPPORTED;
    }
    if (st) {
        st->iters = inner_total;
        st->outer_iters = outer;
        st->fp64_applies = applies64;
        st->status = status;
        st->rel_res_recursive = res;
    }
    return FGH_OK;
}


// ------------------------------------------------------------------------------------------
// Allocation-free application of C = G A (fgh_apply_noalloc): the device buffers of the passes
// (twiddle tables, the two half-spectrum buffers, the last pass's partial sums and a scalar
// block) are carved out of a file-scope device array instead of a caller's workspace.  Each GPU
// holds its own copy of the array for the life of the process, and every call on that GPU
// shares it.  In host code `scratch` only names the array: its device address on the current
// device comes from hipGetSymbolAddress, taken once per device and kept.
// ------------------------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[kScratchDevices] = {};

}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

fgh_status scratch_address(char** out)
{
    int dev = -1;
    HIPOK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return FGH_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FGH_E_DEVICE;
        g_scratch_addr[dev] = static_cast<char*>(ptr);
    }
    *out = g_scratch_addr[dev];
    return FGH_OK;
}

// Offsets of the allocation-free apply's buffers inside the scratch array (256-byte aligned).
struct ScratchLayout {
    size_t tw[3], SA, SB, partials, scalars, total;
};

ScratchLayout scratch_layout(const Geo& g)
{
    ScratchLayout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    for (int a = 0; a < g.d; a++) l.tw[a] = take((size_t)g.L[a] * 16);
    const long long sp = std::max(g.s1, g.s2);
    l.SA = take((size_t)g.d * sp * 16);
    l.SB = take(g.d == 3 ? (size_t)g.d * sp * 16 : 0);  // 2D transforms in place in SA
    l.partials = take(((size_t)g.rows + 64) * 8);         // at most one per row of the last pass
    l.scalars = take(sizeof(Scalars));
    l.total = off;
    return l;
}

// ------------------------------------------------------------------------------------------
// Batches: FP32-refined solves of one shape whose inner FP32 loops share launches.  Each member
// keeps its own plan, buffers, loop scalars and partial sums; its outer FP64 steps are the
// plan's own (solve_one_refined); its inner loop bodies run in batched launches whose
// per-member arithmetic is that of the plan alone, so every member's iterates, counts and
// results are those of fgh_solve on its plan.
// ------------------------------------------------------------------------------------------
struct BatchMember {
    fgh_plan p = nullptr;
    int index = 0;        // position in the caller's arrays
    const double* E = nullptr;  // load (host [d])
    double tol = 0.0;
    double* e = nullptr;  // device [d][grid]
    double normE = 0.0, normb = 0.0, rr = 0.0, res = 0.0, dnorm = 0.0;
    int outer = 0, inner = 0, applies = 0, status = FGH_OK;
    bool done = false;    // stopping test met
    bool active = true;   // still iterating
    bool restored = false; // the plan has its own streams back (it may have been released)
    double eta = 0.0;     // inner relative tolerance of the current outer step
};

// Plans whose loop bodies can share launches: same grid, rule, precision and launch configuration.
bool same_launch_shape(fgh_plan a, fgh_plan b)
{
    if (a->d != b->d || a->rule != b->rule || a->prec != b->prec) return false;
    for (int k = 0; k < 3; k++)
        if (a->N[k] != b->N[k]) return false;
    const OpPlan& x = a->op32;
    const OpPlan& y = b->op32;
    return x.rpb == y.rpb && x.rpb_first == y.rpb_first && x.rpb_fused == y.rpb_fused && x.P_axis == y.P_axis &&
           x.P_mid == y.P_mid && x.mid_pad == y.mid_pad && x.lds_first_v2 == y.lds_first_v2 &&
           x.lds_last_v2 == y.lds_last_v2 && x.lds_fused == y.lds_fused && x.lds_axis == y.lds_axis &&
           x.lds_mid == y.lds_mid && x.v2_row == y.v2_row && x.v2_axis == y.v2_axis && x.v2_mid == y.v2_mid;
}

// Copies the members' argument blocks into the lead plan's table region (one upload per inner
// solve; the tables do not change between loop bodies: the loop's scalars live on the device).
fgh_status upload_tables(fgh_plan lead, int nb, const std::vector<ApplyBundle<float>>& bu,
                         const std::vector<ReduceArgs>& r1, const std::vector<ReduceArgs>& r2,
                         const std::vector<UpdateArgs<float>>& up, hipStream_t s, BatchTables<float>* dev)
{
    std::vector<char> host(kBatchSlabBytes, 0);
    BatchTables<float> h = batch_tables<float>(host.data());
    *dev = batch_tables<float>(lead->ws + lead->lay.slab);
    for (int k = 0; k < nb; k++) {
        h.fa[k] = bu[k].fa;
        h.xf[k] = bu[k].xf;
        h.xi[k] = bu[k].xi;
        h.ma[k] = bu[k].ma;
        h.la[k] = bu[k].la;
        if (!r1.empty()) h.red[k] = r1[k];
        if (!r2.empty()) h.red2[k] = r2[k];
        if (!up.empty()) h.upd[k] = up[k];
    }
    HIPOK(hipMemcpyAsync(lead->ws + lead->lay.slab, host.data(), h.bytes, hipMemcpyHostToDevice, s));
    HIPOK(hipStreamSynchronize(s));  // the host image is released on return
    return FGH_OK;
}

// Loop bodies of a batch in chunks, as run_loop does for one plan (graph replay when the stream
// can be captured); the device stops each member by its own test; returns when all have stopped,
// with each member's count, test quantity (relative to scale[k]) and status.
template <typename Body>
fgh_status run_loop_batch(fgh_plan lead, const std::vector<BatchMember*>& A, hipStream_t s, Body body, uint64_t key,
                          const std::vector<double>& scale, std::vector<SolveOut>* outs)
{
    const bool use_graph = graphs_enabled() && s != nullptr;
    if (use_graph && (lead->gkey != key || !lead->gexec)) {
        drop_graph(lead);
        HIPOK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t ce = hipSuccess;
        for (int k = 0; k < kGraphBodies && ce == hipSuccess; k++) ce = body();
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(s, &g);
        if (ce != hipSuccess || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return FGH_E_DEVICE;
        }
        lead->graph = g;
        HIPOK(hipGraphInstantiate(&lead->gexec, g, nullptr, nullptr, 0));
        lead->gkey = key;
    }
    const int nb = (int)A.size();
    int chunk = 1;
    for (;;) {
        for (int k = 0; k < chunk; k++) {
            if (use_graph) {
                HIPOK(hipGraphLaunch(lead->gexec, s));
            } else {
                for (int b = 0; b < kGraphBodies; b++) HIPOK(body());
            }
        }
        for (int k = 0; k < nb; k++)
            HIPOK(hipMemcpyAsync(A[k]->p->host_buf, A[k]->p->op32.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIPOK(hipStreamSynchronize(s));
        bool all = true;
        for (int k = 0; k < nb; k++) all = all && reinterpret_cast<const Scalars*>(A[k]->p->host_buf)->done != 0;
        if (all) break;
        if (chunk < 4) chunk *= 2;
    }
    outs->assign(nb, SolveOut{});
    for (int k = 0; k < nb; k++) {
        const Scalars* h = reinterpret_cast<const Scalars*>(A[k]->p->host_buf);
        SolveOut& o = (*outs)[k];
        o.iters = h->m;
        o.res = scale[k] > 0 ? h->last / scale[k] : h->last;
        o.status = h->done == 3 ? FGH_E_DIVERGED : h->done == 2 ? FGH_E_NO_CONVERGENCE : FGH_OK;
    }
    return FGH_OK;
}

uint64_t batch_key(uint64_t kind, const std::vector<BatchMember*>& A)
{
    uint64_t h = key_of({kind, (uint64_t)A.size()});
    for (const BatchMember* m : A) h = mix_key(h, bits(m->p));
    return h;
}

// The inner FP32 CG solves C delta = r32 of the active members (cg_core's set-up per member,
// then bodies in shared launches).
fgh_status cg_inner_batch(const std::vector<BatchMember*>& A, int max_iter, hipStream_t s, std::vector<SolveOut>* outs)
{
    const int nb = (int)A.size();
    std::vector<ApplyBundle<float>> bu(nb);
    std::vector<ReduceArgs> r1(nb), r2(nb);
    std::vector<UpdateArgs<float>> up(nb);
    std::vector<double> scale(nb);
    for (int k = 0; k < nb; k++) {
        fgh_plan p = A[k]->p;
        const OpPlan& op = p->op32;
        const long long n = (long long)p->d * p->g.npts;
        const double S = (double)p->g.npts;
        HIPOK(run_copy<float>(s, n, p->p32, p->r32));
        double bb = 0.0;
        int nbk = 0;
        HIPOK(run_dot<float>(op, n, p->r32, p->r32, &nbk));
        fgh_status st = reduce_read(p, op, nbk, RED_TOTAL, &bb);
        if (st) return st;
        scale[k] = std::sqrt(bb / S);
        HIPOK(run_init_loop(op, bb, 0.0, 0.0, A[k]->eta * scale[k], S, 0.0, 0.0, 0.0, max_iter));
        ApplyArgs a;
        a.op = OP_AP_CG;
        a.p_cg = p->p32;
        a.r_cg = p->r32;
        a.epi = EPI_CG;
        a.eq = p->q32;
        a.ep = p->p32;
        a.loop = true;
        HIPOK(build_bundle<float>(op, a, &bu[k]));
        r1[k] = ReduceArgs{op.partials, (int)bu[k].nblk_last, op.sc};
        r2[k] = ReduceArgs{op.partials, vec_blocks(), op.sc};
        up[k] = UpdateArgs<float>{n, p->x32, p->r32, p->p32, p->q32, op.sc, op.partials};
    }
    BatchTables<float> t;
    fgh_plan lead = A[0]->p;
    fgh_status st = upload_tables(lead, nb, bu, r1, r2, up, s, &t);
    if (st) return st;
    const OpPlan& op0 = lead->op32;
    auto body = [&]() -> hipError_t {
        hipError_t e = run_apply_batch<float>(op0, bu[0], t, nb);
        if (e != hipSuccess) return e;
        if ((e = run_reduce_batch(s, t.red, nb, RED_CG_ALPHA)) != hipSuccess) return e;
        if ((e = run_cg_update_batch<float>(s, t.upd, nb)) != hipSuccess) return e;
        return run_reduce_batch(s, t.red2, nb, RED_CG_END);
    };
    return run_loop_batch(lead, A, s, body, batch_key(21, A), scale, outs);
}

// The inner FP32 Eyre-Milton correction solves of the active members (em_core's correction
// form: delta = (A + wI)^{-1}(I - 2G^)(A - wI) delta + r32 from delta = 0), fused bodies.
fgh_status em_inner_batch(const std::vector<BatchMember*>& A, int max_iter, hipStream_t s, std::vector<SolveOut>* outs)
{
    const int nb = (int)A.size();
    std::vector<ApplyBundle<float>> pro(nb), bu(nb);
    std::vector<ReduceArgs> r1(nb);
    std::vector<double> scale(nb);
    bool defer = false;
    for (int k = 0; k < nb; k++) {
        fgh_plan p = A[k]->p;
        const OpPlan& op = p->op32;
        const double S = (double)p->g.npts;
        const double omega = std::sqrt(p->cA * p->CA);
        scale[k] = A[k]->dnorm;
        HIPOK(run_init_loop(op, 0.0, 0.0, 0.0, A[k]->eta * A[k]->dnorm, S, 1e12 * (A[k]->dnorm > 0 ? A[k]->dnorm : 1.0),
                            0.0, 0.0, max_iter));
        if (!fuse_loop(p, op)) return FGH_E_UNSUPPORTED;
        ApplyArgs a;
        a.op = OP_EM;
        a.x = p->x32;
        a.omega = omega;
        a.mult = MULT_EM;
        a.epi = EPI_EM;
        a.ex = p->x32;
        a.src = p->r32;
        for (int c = 0; c < p->d; c++) a.E[c] = A[k]->E[c];
        a.loop = true;
        ApplyArgs ap = a;  // the loop's prologue: the first body's first pass alone
        ap.first_only = true;
        ap.loop = false;
        HIPOK(build_bundle<float>(op, ap, &pro[k]));
        a.skip_first = true;
        a.next_op = OP_EM;
        defer = defer_reduction(op, true);
        a.defer_redop = defer ? RED_STEP_END : -1;
        HIPOK(build_bundle<float>(op, a, &bu[k]));
        bu[k].fa = pro[k].fa;  // the body skips its first pass: the table slot holds the prologue's
        r1[k] = ReduceArgs{op.partials, (int)bu[k].nblk_last, op.sc};
    }
    BatchTables<float> t;
    fgh_plan lead = A[0]->p;
    fgh_status st = upload_tables(lead, nb, bu, r1, {}, {}, s, &t);
    if (st) return st;
    const OpPlan& op0 = lead->op32;
    HIPOK(run_apply_batch<float>(op0, pro[0], t, nb));
    auto body = [&]() -> hipError_t {
        hipError_t e = run_apply_batch<float>(op0, bu[0], t, nb);
        if (e != hipSuccess || defer) return e;
        return run_reduce_batch(s, t.red, nb, RED_STEP_END);
    };
    return run_loop_batch(lead, A, s, body, batch_key(defer ? 23 : 22, A), scale, outs);
}

// rel_res_true of a finished member (as solve_common reports it) and its stats.
fgh_status finish_member(BatchMember* m, fgh_stats* st, double seconds)
{
    fgh_plan p = m->p;
    st->iters = m->inner;
    st->outer_iters = m->outer;
    st->fp64_applies = m->applies;
    st->status = m->status;
    st->rel_res_recursive = m->res;
    st->seconds = seconds;
    st->c_A = p->cA;
    st->C_A = p->CA;
    double bb = 0.0;
    fgh_status s = rhs<double>(p, m->E, p->r64, &bb, nullptr);
    if (s) return s;
    double rt = 0.0;
    if ((s = true_residual(p, m->E, m->e, bb, &rt))) return s;
    st->rel_res_true = rt;
    return FGH_OK;
}

// The outer FP64 defect-correction steps of solve_one_refined for every member in lockstep, with
// the inner solves of the members still iterating batched.  retire(k) is called for member k as
// soon as its result is final.
fgh_status refined_batch(std::vector<BatchMember>& ms, fgh_solver solver, int max_iter, hipStream_t s,
                         fgh_stats* stats, const std::function<void(int)>& retire)
{
    const auto t0 = std::chrono::steady_clock::now();
    // a finished member gets its own streams back before it is retired: the retire callback may
    // release its plan, and nothing here touches it afterwards
    auto finish = [&](BatchMember& m) -> fgh_status {
        if (solver == FGH_EYRE_MILTON) {  // the fluctuation x - E
            fgh_plan p = m.p;
            const long long n = (long long)p->d * p->g.npts;
            double negE[3] = {-m.E[0], -m.E[1], p->d == 3 ? -m.E[2] : 0.0};
            HIPOK(run_fill_field<double>(s, p->d, p->g.npts, p->q64, negE));
            HIPOK(run_add_f64(s, n, m.e, p->q64));
        }
        if (m.status == FGH_OK && !m.done) m.status = FGH_E_NO_CONVERGENCE;
        m.active = false;
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        fgh_stats st{};
        fgh_status r = finish_member(&m, &st, secs);
        if (r) return r;
        HIPOK(hipStreamSynchronize(s));
        if (stats) stats[m.index] = st;
        m.p->stream = m.p->op64.stream = m.p->op32.stream = m.p->caller;
        m.restored = true;
        if (retire) retire(m.index);
        return FGH_OK;
    };
    const int outer_cap = solver == FGH_EYRE_MILTON ? 200 : 64;
    // set-up per member (solve_one_refined's first steps)
    for (BatchMember& m : ms) {
        fgh_plan p = m.p;
        const long long n = (long long)p->d * p->g.npts;
        const double S = (double)p->g.npts;
        for (int c = 0; c < p->d; c++) m.normE += m.E[c] * m.E[c];
        m.normE = std::sqrt(m.normE);
        if (solver == FGH_EYRE_MILTON) {
            HIPOK(run_fill_field<double>(s, p->d, p->g.npts, m.e, m.E));  // x = E
        } else {
            HIPOK(run_fill<double>(s, n, m.e, 0.0));
            double bb = 0.0, ae2 = 0.0;
            fgh_status st = rhs<double>(p, m.E, p->r64, &bb, &ae2);
            if (st) return st;
            m.applies++;
            const bool zero = !(std::sqrt(bb / S) > kZeroRhs * std::sqrt(ae2 / S));
            m.normb = std::sqrt(bb / S);
            m.rr = bb;
            if (zero) {
                m.done = true;
                fgh_status r = finish(m);
                if (r) return r;
            }
        }
    }
    for (int outer = 0; outer < outer_cap; outer++) {
        std::vector<BatchMember*> A;
        for (BatchMember& m : ms) {
            if (!m.active) continue;
            fgh_plan p = m.p;
            const long long n = (long long)p->d * p->g.npts;
            const double S = (double)p->g.npts;
            m.outer = outer;
            fgh_status st;
            if (solver == FGH_EYRE_MILTON) {
                const double omega = std::sqrt(p->cA * p->CA);
                HIPOK(run_copy<double>(s, n, p->r64, m.e));
                ApplyArgs a;
                a.op = OP_EM;
                a.x = p->r64;
                a.omega = omega;
                a.mult = MULT_EM;
                a.epi = EPI_EM;
                a.ex = p->r64;
                for (int c = 0; c < p->d; c++) a.E[c] = m.E[c];
                int nbk = 0;
                HIPOK(run_apply<double>(p->op64, a, &nbk));
                m.applies++;
                double dd;
                if ((st = reduce_read(p, p->op64, nbk, RED_TOTAL, &dd))) return st;
                m.dnorm = std::sqrt(dd / S);
                m.res = m.normE > 0 ? m.dnorm / m.normE : m.dnorm;
                if (!std::isfinite(m.dnorm) || m.dnorm > 1e12 * (m.normE > 0 ? m.normE : 1.0)) {
                    m.status = FGH_E_DIVERGED;
                    if ((st = finish(m))) return st;
                    continue;
                }
                if (m.dnorm <= m.tol * m.normE) {
                    HIPOK(run_copy<double>(s, n, m.e, p->r64));
                    m.done = true;
                    if ((st = finish(m))) return st;
                    continue;
                }
                HIPOK(run_axpby(s, n, p->q64, 1.0, p->r64, 0.0));
                HIPOK(run_axpby(s, n, p->q64, -1.0, m.e, 1.0));
                HIPOK(run_f64_to_f32(s, n, p->r32, p->q64));
                HIPOK(run_fill<float>(s, n, p->x32, 0.0f));
                m.eta = std::max(m.tol * m.normE / m.dnorm, kInnerTolMin);
            } else {
                if (outer > 0) {
                    ApplyArgs a;
                    a.op = OP_AX;
                    a.x = m.e;
                    for (int c = 0; c < p->d; c++) a.E[c] = m.E[c];
                    a.epi = EPI_STORE;
                    a.sgn = -1.0;
                    a.y = p->r64;
                    int nbk = 0;
                    HIPOK(run_apply<double>(p->op64, a, &nbk));
                    m.applies++;
                    if ((st = reduce_read(p, p->op64, nbk, RED_TOTAL, &m.rr))) return st;
                }
                m.res = std::sqrt(m.rr / S) / m.normb;
                if (!std::isfinite(m.rr)) {
                    m.status = FGH_E_DIVERGED;
                    if ((st = finish(m))) return st;
                    continue;
                }
                if (m.res <= m.tol) {
                    m.done = true;
                    if ((st = finish(m))) return st;
                    continue;
                }
                m.eta = std::max(m.tol / m.res, kInnerTolMin);
                HIPOK(run_f64_to_f32(s, n, p->r32, p->r64));
                HIPOK(run_fill<float>(s, n, p->x32, 0.0f));
            }
            A.push_back(&m);
        }
        if (A.empty()) break;
        for (size_t c = 0; c < A.size(); c += kMaxBatch) {
            std::vector<BatchMember*> G(A.begin() + c, A.begin() + std::min(A.size(), c + kMaxBatch));
            std::vector<SolveOut> outs;
            fgh_status st = solver == FGH_EYRE_MILTON ? em_inner_batch(G, max_iter, s, &outs)
                                                      : cg_inner_batch(G, max_iter, s, &outs);
            if (st) return st;
            for (size_t k = 0; k < G.size(); k++) {
                BatchMember& m = *G[k];
                fgh_plan p = m.p;
                const long long n = (long long)p->d * p->g.npts;
                m.inner += outs[k].iters;
                if (outs[k].status == FGH_E_DIVERGED) {
                    m.status = FGH_E_DIVERGED;
                    if ((st = finish(m))) return st;
                    continue;
                }
                if (solver == FGH_EYRE_MILTON) {
                    HIPOK(run_add_f32_to_f64(s, n, m.e, p->x32));
                } else {
                    // x += G delta in FP64
                    HIPOK(run_fill<double>(s, n, p->p64, 0.0));
                    HIPOK(run_add_f32_to_f64(s, n, p->p64, p->x32));
                    ApplyArgs a;
                    a.op = OP_ID;
                    a.x = p->p64;
                    a.epi = EPI_STORE;
                    a.sgn = 1.0;
                    a.y = p->q64;
                    int nbk = 0;
                    HIPOK(run_apply<double>(p->op64, a, &nbk));
                    m.applies++;
                    HIPOK(run_add_f64(s, n, m.e, p->q64));
                }
            }
        }
    }
    for (BatchMember& m : ms)
        if (m.active) {
            m.outer = outer_cap;
            fgh_status st = finish(m);
            if (st) return st;
        }
    return FGH_OK;
}


// Symmetric tridiagonal matrix with diagonal a and off-diagonal b: the number of its eigenvalues
// below x, from the signs of the pivots of the LDL^T factorisation of T - x I (Sturm sequence;
// a zero pivot is replaced by a tiny negative one, as in the bisection method of Barth, Martin
// and Wilkinson, 1967).
int tridiag_count_below(const std::vector<double>& a, const std::vector<double>& b, double x, double pivmin)
{
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < a.size(); i++) {
        q = a[i] - x - (i ? b[i - 1] * b[i - 1] / q : 0.0);
        if (std::fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) cnt++;
    }
    return cnt;
}

// The k-th smallest eigenvalue (k from 0) of that matrix by bisection inside its Gershgorin
// interval, to the resolution of double precision.
double tridiag_eigenvalue(const std::vector<double>& a, const std::vector<double>& b, int k)
{
    const size_t m = a.size();
    double lo = a[0], hi = a[0], scale = 0.0;
    for (size_t i = 0; i < m; i++) {
        const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
        scale = std::max(scale, std::fabs(a[i]) + r);
    }
    const double pivmin = std::max(scale, 1e-300) * 1e-300;
    for (int it = 0; it < 2000; it++) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (tridiag_count_below(a, b, mid, pivmin) > k)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

}  // namespace

extern "C" {

const char* fgh_status_string(fgh_status s)
{
    switch (s) {
        case FGH_OK: return "ok";
        case FGH_E_INVALID: return "invalid argument";
        case FGH_E_NOT_SPD: return "coefficients not symmetric positive definite";
        case FGH_E_UNSUPPORTED: return "unsupported combination";
        case FGH_E_WORKSPACE: return "workspace missing or too small";
        case FGH_E_NO_CONVERGENCE: return "no convergence within the iteration cap";
        case FGH_E_DIVERGED: return "diverged";
        case FGH_E_DEVICE: return "HIP runtime error";
        case FGH_E_CANCELLED: return "request cancelled";
    }
    return "unknown status";
}

fgh_status fgh_plan_workspace(int d, const int32_t* N, fgh_rule rule, fgh_precision precision, fgh_akind a_kind,
                              size_t* bytes)
{
    if (!bytes) return FGH_E_INVALID;
    if (rule != FGH_GANI && rule != FGH_GA) return FGH_E_INVALID;
    if (precision != FGH_FP64 && precision != FGH_FP32_REFINED) return FGH_E_INVALID;
    if (a_kind < FGH_A_SYM || a_kind > FGH_A_PHASE) return FGH_E_INVALID;
    Geo g;
    if (!make_geo(d, N, rule, &g)) return FGH_E_INVALID;
    *bytes = make_layout(g, N, rule, precision, a_kind).total;
    return FGH_OK;
}

fgh_status fgh_plan_create(fgh_plan* out, int d, const int32_t* N, fgh_rule rule, fgh_precision precision,
                           fgh_akind a_kind, const void* A, const uint8_t* phase, const double* phase_table,
                           int n_phases, double c_A, double C_A, void* workspace, size_t workspace_bytes,
                           void* stream)
{
    if (!out) return FGH_E_INVALID;
    *out = nullptr;
    size_t need = 0;
    fgh_status s = fgh_plan_workspace(d, N, rule, precision, a_kind, &need);
    if (s) return s;
    if (a_kind == FGH_A_PHASE) {
        if (!phase || !phase_table || n_phases < 1 || n_phases > kMaxPhases) return FGH_E_INVALID;
    } else if (!A) {
        return FGH_E_INVALID;
    }
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) % kAlign)) return FGH_E_WORKSPACE;
    fgh_plan p = new (std::nothrow) fgh_plan_s();
    if (!p) return FGH_E_DEVICE;
    p->d = d;
    for (int a = 0; a < 3; a++) p->N[a] = a < d ? N[a] : 1;
    p->rule = rule;
    p->prec = precision;
    p->akind = a_kind;
    make_geo(d, N, rule, &p->g);
    p->lay = make_layout(p->g, N, rule, precision, a_kind);
    p->ws = static_cast<char*>(workspace);
    p->stream = static_cast<hipStream_t>(stream);
    p->caller = p->stream;
    p->ncoef_op = (a_kind == FGH_A_SYM) ? ncoef_for(d) : 1;
    if (hipHostMalloc(reinterpret_cast<void**>(&p->host_buf), 64 * sizeof(double)) != hipSuccess) {
        delete p;
        return FGH_E_DEVICE;
    }
    if (hipStreamCreateWithFlags(&p->sstream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipHostFree(p->host_buf);
        delete p;
        return FGH_E_DEVICE;
    }
    auto fail = [&](fgh_status e) {
        fgh_plan_destroy(p);
        return e;
    };
    const int nc = ncoef_for(d);
    p->nphase = a_kind == FGH_A_PHASE ? n_phases : 0;
    for (int i = 0; i < kMaxPhases; i++)
        for (int q = 0; q < 6; q++) p->tab[i][q] = (i < p->nphase && q < nc) ? phase_table[i * nc + q] : 0.0;
    if (a_kind == FGH_A_PHASE)
        for (int i = 0; i < p->nphase; i++)
            for (int q = 0; q < nc; q++)
                if (!std::isfinite(p->tab[i][q])) return fail(FGH_E_NOT_SPD);
    fill_opplan(p, &p->op64, false);
    fill_opplan(p, &p->op32, true);
    const long long nv = (long long)d * p->g.npts;
    double* v64 = reinterpret_cast<double*>(p->ws + p->lay.vec64);
    p->r64 = v64;
    p->p64 = v64 + nv;
    p->q64 = v64 + 2 * nv;
    float* v32 = reinterpret_cast<float*>(p->ws + p->lay.vec32);
    p->x32 = v32;
    p->r32 = v32 + nv;
    p->p32 = v32 + 2 * nv;
    p->q32 = v32 + 3 * nv;
    if ((s = upload_twiddles(p))) return fail(s);
    // the tile timings below run the passes on the spectrum buffers, on the vector storage (as a
    // third spectrum) and on r64 / r32: give them defined values (zeros and ones) instead of what
    // the workspace held before
    {
        const long long sp = std::max(p->g.s1, p->g.s2);
        if (run_fill<double>(p->stream, 2 * d * sp, reinterpret_cast<double*>(p->ws + p->lay.SA), 0.0) != hipSuccess ||
            run_fill<double>(p->stream, 2 * d * sp, reinterpret_cast<double*>(p->ws + p->lay.SB), 0.0) != hipSuccess ||
            run_fill<double>(p->stream, std::max(3 * nv, 2 * d * sp), v64, 0.0) != hipSuccess ||
            run_fill<double>(p->stream, nv, p->r64, 1.0) != hipSuccess ||
            (precision == FGH_FP32_REFINED && (run_fill<float>(p->stream, 4 * nv, v32, 0.0f) != hipSuccess ||
                                               run_fill<float>(p->stream, nv, p->r32, 1.0f) != hipSuccess)))
            return fail(FGH_E_DEVICE);
    }
    if ((s = tune_middle(p, &p->op64, false))) return fail(s);
    if (precision == FGH_FP32_REFINED && (s = tune_middle(p, &p->op32, true))) return fail(s);
    if ((s = tune_axis(p, &p->op64, false))) return fail(s);
    if (precision == FGH_FP32_REFINED && (s = tune_axis(p, &p->op32, true))) return fail(s);
    if ((s = tune_first(p, &p->op64, false, p->r64))) return fail(s);
    if (precision == FGH_FP32_REFINED && (s = tune_first(p, &p->op32, true, p->r32))) return fail(s);

    long long nN = 1;
    for (int a = 0; a < d; a++) nN *= N[a];
    double* partials = reinterpret_cast<double*>(p->ws + p->lay.partials);

    // spectral bounds of the input (eq:A)
    double lo = 1e300, hi = -1e300;
    if (a_kind == FGH_A_PHASE) {
        unsigned* mask = reinterpret_cast<unsigned*>(p->ws + p->lay.mask);
        if (run_fill<unsigned>(p->stream, 1, mask, 0u) != hipSuccess) return fail(FGH_E_DEVICE);
        if (run_phase_mask(p->stream, phase, nN, mask) != hipSuccess) return fail(FGH_E_DEVICE);
        unsigned hm = 0;
        if (hipMemcpyAsync(&hm, mask, sizeof(unsigned), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
            hipStreamSynchronize(p->stream) != hipSuccess)
            return fail(FGH_E_DEVICE);
        if (hm >> p->nphase) return fail(FGH_E_INVALID);  // a phase index outside the table
        for (int i = 0; i < p->nphase; i++)
            if (hm & (1u << i)) {
                double l, h;
                host_sym_eigs(d, p->tab[i], &l, &h);
                lo = std::fmin(lo, l);
                hi = std::fmax(hi, h);
            }
    } else {
        int nb = 0;
        if (run_eig_bounds(p->stream, d, a_kind == FGH_A_ISO ? AK_ISO : AK_SYM, static_cast<const double*>(A), nN,
                           partials, &nb) != hipSuccess)
            return fail(FGH_E_DEVICE);
        double lh[2];
        if (run_minmax_reduce(p->stream, partials, nb, lh) != hipSuccess) return fail(FGH_E_DEVICE);
        lo = lh[0];
        hi = lh[1];
    }
    if (!(lo > 0.0) || !std::isfinite(hi)) return fail(FGH_E_NOT_SPD);
    if (c_A > 0.0 && C_A > 0.0) {
        if (c_A > C_A) return fail(FGH_E_NOT_SPD);
        p->cA = c_A;
        p->CA = C_A;
    } else {
        p->cA = lo;
        p->CA = hi;
    }

    // operator coefficients (CoefArgs)
    CoefArgs ca{};
    for (int i = 0; i < kMaxPhases; i++)
        for (int q = 0; q < 6; q++) ca.tab[i][q] = p->tab[i][q];
    const double omega = std::sqrt(p->cA * p->CA);
    for (int i = 0; i < p->nphase; i++) host_shift_inverse(d, p->tab[i], omega, ca.tab_inv[i]);
    const long long npts = p->g.npts;
    if (rule == FGH_GA) {
        GaAsm ga{};
        ga.d = d;
        ga.nN = nN;
        ga.nM = npts;
        std::vector<double> buf;
        for (int a = 0; a < d; a++) {
            ga.N[a] = N[a];
            ga.M[a] = 2 * N[a] - 1;
            // sinc(n / N) for the signed frequencies n of the M positions, and DFT tables
            buf.assign((size_t)ga.M[a], 0.0);
            for (int i = 0; i < ga.M[a]; i++) {
                const int nf = (2 * i < ga.M[a]) ? i : i - ga.M[a];
                if (nf == 0) {
                    buf[i] = 1.0;
                } else {
                    const long double t = 3.141592653589793238462643383279502884L * (long double)nf / (long double)N[a];
                    buf[i] = (double)(sinl(t) / t);
                }
            }
            if (hipMemcpyAsync(p->ws + p->lay.sinc[a], buf.data(), (size_t)ga.M[a] * 8, hipMemcpyHostToDevice, p->stream) != hipSuccess)
                return fail(FGH_E_DEVICE);
            std::vector<double> t;
            for (int which = 0; which < 2; which++) {
                const int L = which ? ga.M[a] : ga.N[a];
                t.assign(2 * (size_t)L, 0.0);
                for (int m = 0; m < L; m++) {
                    const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)L;
                    t[2 * m] = (double)cosl(ang);
                    t[2 * m + 1] = -(double)sinl(ang);
                }
                const size_t off = which ? p->lay.twM[a] : p->lay.twN[a];
                if (hipMemcpyAsync(p->ws + off, t.data(), (size_t)L * 16, hipMemcpyHostToDevice, p->stream) != hipSuccess ||
                    hipStreamSynchronize(p->stream) != hipSuccess)
                    return fail(FGH_E_DEVICE);
            }
            ga.sinc[a] = reinterpret_cast<const double*>(p->ws + p->lay.sinc[a]);
            ga.twN[a] = reinterpret_cast<const double2*>(p->ws + p->lay.twN[a]);
            ga.twM[a] = reinterpret_cast<const double2*>(p->ws + p->lay.twM[a]);
        }
        ga.c0 = reinterpret_cast<double2*>(p->ws + p->lay.vec64);
        ga.c1 = ga.c0 + npts;
        double* coef = reinterpret_cast<double*>(p->ws + p->lay.coef64);
        const int kind = a_kind == FGH_A_PHASE ? AK_PHASE : a_kind == FGH_A_ISO ? AK_ISO : AK_SYM;
        for (int q = 0; q < p->ncoef_op; q++) {
            double pv[kMaxPhases] = {0};
            for (int i = 0; i < p->nphase; i++) pv[i] = p->tab[i][0];  // isotropic phases: a00
            if (run_ga_component(p->stream, ga, kind, static_cast<const double*>(A), q, phase, pv, p->nphase,
                                 coef + q * npts) != hipSuccess)
                return fail(FGH_E_DEVICE);
        }
        if (hipStreamSynchronize(p->stream) != hipSuccess) return fail(FGH_E_DEVICE);
        ca.kind = p->ncoef_op == 1 ? AK_ISO : AK_SYM;
        ca.ncoef = p->ncoef_op;
        ca.coef = coef;
        ca.phase = nullptr;
        if (a_kind == FGH_A_PHASE) {
            // the phase table must be isotropic for the scalar double-grid representation
            for (int i = 0; i < p->nphase; i++) {
                const double* t = p->tab[i];
                const bool iso = d == 2 ? (t[1] == 0.0 && t[0] == t[2])
                                        : (t[1] == 0.0 && t[2] == 0.0 && t[4] == 0.0 && t[0] == t[3] && t[0] == t[5]);
                if (!iso) return fail(FGH_E_UNSUPPORTED);
            }
        }
    } else {
        ca.kind = a_kind == FGH_A_PHASE ? AK_PHASE : a_kind == FGH_A_ISO ? AK_ISO : AK_SYM;
        ca.ncoef = a_kind == FGH_A_SYM ? nc : 1;
        ca.coef = A;
        ca.phase = phase;
    }
    p->op64.A = ca;
    p->op32.A = ca;
    if (precision == FGH_FP32_REFINED && ca.kind != AK_PHASE) {
        float* c32 = reinterpret_cast<float*>(p->ws + p->lay.coef32);
        if (run_to_f32(p->stream, (long long)ca.ncoef * npts, c32, static_cast<const double*>(ca.coef)) != hipSuccess)
            return fail(FGH_E_DEVICE);
        p->op32.A.coef = c32;
    }
    // the fused pass multiplies by A: tuned once the operator's coefficients are in place
    if ((s = tune_fused(p, &p->op64, false, p->r64))) return fail(s);
    if (precision == FGH_FP32_REFINED && (s = tune_fused(p, &p->op32, true, p->r32))) return fail(s);
    if ((s = tune_first_cg(p, &p->op64, false))) return fail(s);
    if (precision == FGH_FP32_REFINED && (s = tune_first_cg(p, &p->op32, true))) return fail(s);
    if (hipStreamSynchronize(p->stream) != hipSuccess) return fail(FGH_E_DEVICE);
    *out = p;
    return FGH_OK;
}

void fgh_plan_destroy(fgh_plan p)
{
    if (!p) return;
    drop_graph(p);
    if (p->sstream) (void)hipStreamDestroy(p->sstream);
    if (p->prof) {
        p->prof->destroy();
        delete p->prof;
    }
    if (p->host_buf) (void)hipHostFree(p->host_buf);
    delete p;
}

int64_t fgh_plan_grid_points(fgh_plan p) { return p ? p->g.npts : 0; }

fgh_status fgh_plan_set_profiling(fgh_plan p, int enable)
{
    if (!p) return FGH_E_INVALID;
    if (enable) {
        if (!p->prof) {
            p->prof = new (std::nothrow) Profiler();
            if (!p->prof) return FGH_E_DEVICE;
        }
        HIPOK(p->prof->init(p->stream));
        p->prof->mask = (unsigned)enable & ((1u << PK_KINDS) - 1u);
        p->op64.prof = p->prof;
        p->op32.prof = p->prof;
    } else {
        p->op64.prof = nullptr;
        p->op32.prof = nullptr;
    }
    return FGH_OK;
}

fgh_status fgh_plan_read_profile(fgh_plan p, double* ms, int64_t* launches)
{
    if (!p || !ms || !launches) return FGH_E_INVALID;
    for (int k = 0; k < PK_KINDS; k++) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    if (!p->prof) return FGH_OK;
    HIPOK(p->prof->drain());
    for (int k = 0; k < PK_KINDS; k++) {
        long long n = 0;
        p->prof->working(k, &ms[k], &n);
        launches[k] = n;
    }
    return FGH_OK;
}

fgh_status fgh_plan_bounds(fgh_plan p, double* c_A, double* C_A)
{
    if (!p || !c_A || !C_A) return FGH_E_INVALID;
    *c_A = p->cA;
    *C_A = p->CA;
    return FGH_OK;
}

fgh_status fgh_apply(fgh_plan p, const double* x, double* y)
{
    if (!p || !x || !y) return FGH_E_INVALID;
    ApplyArgs a;
    a.op = OP_AX;
    a.x = x;
    a.epi = EPI_STORE;
    a.sgn = 1.0;
    a.y = y;
    int nb = 0;
    HIPOK(run_apply<double>(p->op64, a, &nb));
    return FGH_OK;
}

fgh_status fgh_apply_f32(fgh_plan p, const float* x, float* y)
{
    if (!p || !x || !y) return FGH_E_INVALID;
    if (p->prec != FGH_FP32_REFINED) return FGH_E_UNSUPPORTED;
    ApplyArgs a;
    a.op = OP_AX;
    a.x = x;
    a.epi = EPI_STORE;
    a.sgn = 1.0;
    a.y = y;
    int nb = 0;
    HIPOK(run_apply<float>(p->op32, a, &nb));
    return FGH_OK;
}

fgh_status fgh_apply_noalloc(int d, const int32_t* N, fgh_akind a_kind, const void* A, const uint8_t* phase,
                             const double* phase_table, int n_phases, const double* x, double* y, void* stream)
{
    if (!x || !y) return FGH_E_INVALID;
    if (a_kind < FGH_A_SYM || a_kind > FGH_A_PHASE) return FGH_E_INVALID;
    Geo g;
    if (!make_geo(d, N, FGH_GANI, &g)) return FGH_E_INVALID;
    const int nc = ncoef_for(d);
    CoefArgs ca{};
    if (a_kind == FGH_A_PHASE) {
        if (!phase || !phase_table || n_phases < 1 || n_phases > kMaxPhases) return FGH_E_INVALID;
        for (int i = 0; i < n_phases; i++)
            for (int q = 0; q < nc; q++) {
                if (!std::isfinite(phase_table[i * nc + q])) return FGH_E_INVALID;
                ca.tab[i][q] = phase_table[i * nc + q];
            }
        ca.kind = AK_PHASE;
        ca.ncoef = 1;
        ca.coef = nullptr;
        ca.phase = phase;
    } else {
        if (!A) return FGH_E_INVALID;
        ca.kind = a_kind == FGH_A_ISO ? AK_ISO : AK_SYM;
        ca.ncoef = a_kind == FGH_A_SYM ? nc : 1;
        ca.coef = A;
        ca.phase = nullptr;
    }
    const ScratchLayout l = scratch_layout(g);
    if (l.total > kScratchBytes) return FGH_E_WORKSPACE;  // the grid does not fit the scratch array
    char* base = nullptr;
    fgh_status s = scratch_address(&base);
    if (s) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* tw[3] = {nullptr, nullptr, nullptr};
    for (int a = 0; a < d; a++) {
        tw[a] = base + l.tw[a];
        HIPOK(run_twiddles(st, g.L[a], reinterpret_cast<double2*>(tw[a])));
    }
    OpPlan op{};
    fill_opplan_at(&op, g, false, tw, base + l.SA, base + l.SB, reinterpret_cast<double*>(base + l.partials),
                   reinterpret_cast<Scalars*>(base + l.scalars), st);
    op.A = ca;
    ApplyArgs a;
    a.op = OP_AX;
    a.x = x;
    a.epi = EPI_STORE;
    a.sgn = 1.0;
    a.y = y;
    int nb = 0;
    HIPOK(run_apply<double>(op, a, &nb));
    return FGH_OK;
}

fgh_status fgh_ga_coefficients(fgh_plan p, double* out)
{
    if (!p || !out) return FGH_E_INVALID;
    if (p->rule != FGH_GA) return FGH_E_INVALID;
    const size_t bytes = (size_t)p->ncoef_op * p->g.npts * 8;
    HIPOK(hipMemcpyAsync(out, p->ws + p->lay.coef64, bytes, hipMemcpyDeviceToDevice, p->stream));
    HIPOK(hipStreamSynchronize(p->stream));
    return FGH_OK;
}

static fgh_status solve_common(fgh_plan p, fgh_solver solver, const double* E, int nrhs, double tol, int max_iter,
                               int fixed, double* e, fgh_stats* stats)
{
    if (!p || !E || !e || nrhs < 1) return FGH_E_INVALID;
    if (solver < FGH_RICHARDSON || solver > FGH_EYRE_MILTON) return FGH_E_INVALID;
    if (fixed <= 0 && (!(tol > 0.0) || !(tol < 1.0) || max_iter < 1)) return FGH_E_INVALID;
    if (solver == FGH_EYRE_MILTON && p->rule == FGH_GA) return FGH_E_UNSUPPORTED;
    for (int j = 0; j < nrhs * p->d; j++)
        if (!std::isfinite(E[j])) return FGH_E_INVALID;
    const long long n = (long long)p->d * p->g.npts;
    int worst = FGH_OK;
    // Work runs on the plan-internal stream after everything already queued on the caller's.
    if (hipStreamSynchronize(p->caller) != hipSuccess) return FGH_E_DEVICE;
    struct StreamSwap {
        fgh_plan p;
        explicit StreamSwap(fgh_plan q) : p(q)
        {
            p->stream = p->op64.stream = p->op32.stream = p->sstream;
            if (p->prof) p->prof->stream = p->sstream;
        }
        ~StreamSwap()
        {
            (void)hipStreamSynchronize(p->sstream);
            p->stream = p->op64.stream = p->op32.stream = p->caller;
            if (p->prof) p->prof->stream = p->caller;
        }
    } swap_guard(p);
    for (int j = 0; j < nrhs; j++) {
        const double* Ej = E + j * p->d;
        double* ej = e + j * n;
        fgh_stats st{};
        const auto t0 = std::chrono::steady_clock::now();
        fgh_status s;
        if (p->prec == FGH_FP32_REFINED && fixed <= 0)
            s = solve_one_refined(p, solver, Ej, tol, max_iter, ej, &st);
        else
            s = solve_one_fp64(p, solver, Ej, tol, max_iter, fixed, ej, &st, j);
        if (s) return s;
        if (hipStreamSynchronize(p->stream) != hipSuccess) return FGH_E_DEVICE;
        const auto t1 = std::chrono::steady_clock::now();
        st.seconds = std::chrono::duration<double>(t1 - t0).count();
        st.c_A = p->cA;
        st.C_A = p->CA;
        // true residual at exit (not timed)
        double bb = 0.0;
        if ((s = rhs<double>(p, Ej, p->r64, &bb, nullptr))) return s;
        double rt = 0.0;
        if ((s = true_residual(p, Ej, ej, bb, &rt))) return s;
        st.rel_res_true = rt;
        if (stats) stats[j] = st;
        if (st.status != FGH_OK && worst == FGH_OK) worst = st.status;
    }
    return (fgh_status)worst;
}

fgh_status fgh_solve(fgh_plan p, fgh_solver solver, const double* E, int nrhs, double tol, int max_iter, double* e,
                     fgh_stats* stats)
{
    return solve_common(p, solver, E, nrhs, tol, max_iter, 0, e, stats);
}

fgh_status fgh_solve_fixed(fgh_plan p, fgh_solver solver, const double* E, int nrhs, int iters, double* e,
                           fgh_stats* stats)
{
    if (iters < 1) return FGH_E_INVALID;
    if (p && p->prec != FGH_FP64) return FGH_E_UNSUPPORTED;
    return solve_common(p, solver, E, nrhs, 0.5, iters, iters, e, stats);
}

}  // extern "C"

namespace fgh {
bool batching_enabled()
{
    const char* v = std::getenv("FGH_BATCH");
    return !(v && v[0] == '0');
}

double phase_table_contrast(int d, const double* table, int n_phases)
{
    const int nc = d == 2 ? 3 : 6;
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < n_phases; i++) {
        double l = 0.0, h = 0.0;
        host_sym_eigs(d, table + (size_t)i * nc, &l, &h);
        lo = i ? std::min(lo, l) : l;
        hi = i ? std::max(hi, h) : h;
    }
    return lo > 0.0 && std::isfinite(hi) ? hi / lo : 0.0;
}

bool batch_shares_launches(int d, const int32_t* N, int rule, int precision, int solver)
{
    if (!batching_enabled()) return false;
    if (precision != FGH_FP32_REFINED || (solver != FGH_CG && solver != FGH_EYRE_MILTON)) return false;
    if (solver == FGH_EYRE_MILTON && rule == FGH_GA) return false;
    Geo g;
    if (!make_geo(d, N, rule, &g)) return false;
    const Config c = choose_config(g, 8, 4);
    return c.v2_row && c.v2_mid && (d == 2 || c.v2_axis);
}
}  // namespace fgh

extern "C" {

fgh_status fgh_solve_batch(fgh_plan* plans, int n, fgh_solver solver, const double* E, const double* tol,
                           int max_iter, double* const* e, fgh_stats* stats, fgh_retire_fn retire, void* user)
{
    if (!plans || n < 1 || n > 64 || !E || !tol || !e) return FGH_E_INVALID;
    if (solver < FGH_RICHARDSON || solver > FGH_EYRE_MILTON || max_iter < 1) return FGH_E_INVALID;
    for (int k = 0; k < n; k++) {
        fgh_plan p = plans[k];
        if (!p || !e[k] || !(tol[k] > 0.0) || !(tol[k] < 1.0)) return FGH_E_INVALID;
        if (p->d != plans[0]->d || p->rule != plans[0]->rule || p->prec != plans[0]->prec) return FGH_E_INVALID;
        for (int a = 0; a < 3; a++)
            if (p->N[a] != plans[0]->N[a]) return FGH_E_INVALID;
        for (int c = 0; c < p->d; c++)
            if (!std::isfinite(E[k * p->d + c])) return FGH_E_INVALID;
        for (int j = 0; j < k; j++)
            if (plans[j] == p) return FGH_E_INVALID;  // members must not share buffers
    }
    if (solver == FGH_EYRE_MILTON && plans[0]->rule == FGH_GA) return FGH_E_UNSUPPORTED;
    const int d = plans[0]->d;
    // a single member runs as fgh_solve (the shared-launch driver's tables and per-member graphs
    // only pay when launches are shared)
    bool shared = n > 1 && plans[0]->prec == FGH_FP32_REFINED && (solver == FGH_CG || solver == FGH_EYRE_MILTON) &&
                  batchable(plans[0]->op32) && fgh::batching_enabled();
    for (int k = 0; k < n && shared; k++)
        shared = same_launch_shape(plans[0], plans[k]) && !plans[k]->hist_fn && !plans[k]->op32.prof &&
                 !plans[k]->op64.prof;
    int worst = FGH_OK;
    if (!shared) {
        // one member after another, each exactly as fgh_solve
        for (int k = 0; k < n; k++) {
            fgh_stats st{};
            const fgh_status s = solve_common(plans[k], solver, E + k * d, 1, tol[k], max_iter, 0, e[k], &st);
            if (s && s != FGH_E_NO_CONVERGENCE && s != FGH_E_DIVERGED) return s;
            if (stats) stats[k] = st;
            if (st.status != FGH_OK && worst == FGH_OK) worst = st.status;
            if (retire) retire(user, k);
        }
        return (fgh_status)worst;
    }
    for (int k = 0; k < n; k++)
        if (hipStreamSynchronize(plans[k]->caller) != hipSuccess) return FGH_E_DEVICE;
    // every member's work runs on the first member's internal stream (capturable); members that
    // were not retired get their streams back on every way out
    hipStream_t s = plans[0]->sstream;
    std::vector<BatchMember> ms(n);
    struct Swap {
        std::vector<BatchMember>& ms;
        hipStream_t s;
        ~Swap()
        {
            (void)hipStreamSynchronize(s);
            for (BatchMember& m : ms)
                if (!m.restored && m.p) m.p->stream = m.p->op64.stream = m.p->op32.stream = m.p->caller;
        }
    } swap{ms, s};
    for (int k = 0; k < n; k++) plans[k]->stream = plans[k]->op64.stream = plans[k]->op32.stream = s;
    for (int k = 0; k < n; k++) {
        ms[k].p = plans[k];
        ms[k].index = k;
        ms[k].E = E + k * d;
        ms[k].tol = tol[k];
        ms[k].e = e[k];
    }
    std::function<void(int)> rf;
    if (retire) rf = [retire, user](int k) { retire(user, k); };
    const fgh_status st = refined_batch(ms, solver, max_iter, s, stats, rf);
    if (st) return st;
    for (const BatchMember& m : ms)
        if (m.status != FGH_OK && worst == FGH_OK) worst = m.status;
    return (fgh_status)worst;
}

fgh_status fgh_effective(fgh_plan p, const double* E, int nrhs, const double* e, double* bilinear, double* flux)
{
    if (!p || !E || !e || nrhs < 1 || nrhs > 3) return FGH_E_INVALID;
    const int d = p->d;
    // loads into the scalar block (device) for the kernel
    double* Ed = reinterpret_cast<Scalars*>(p->ws + p->lay.scalars)->aux;
    HIPOK(hipMemcpyAsync(Ed, E, sizeof(double) * nrhs * d, hipMemcpyHostToDevice, p->stream));
    int nb = 0;
    HIPOK(run_effective(p->op64, nrhs, Ed, e, &nb));
    const int nv = nrhs * nrhs + nrhs * d;
    double host[18];
    HIPOK(run_reduce_multi(p->op64, nb, nv, host));
    const double S = (double)p->g.npts;
    if (bilinear)
        for (int q = 0; q < nrhs * nrhs; q++) bilinear[q] = host[q] / S;
    if (flux)
        for (int q = 0; q < nrhs * d; q++) flux[q] = host[nrhs * nrhs + q] / S;
    return FGH_OK;
}

fgh_status fgh_plan_set_history(fgh_plan p, double* res_hist, double* energy_hist, double* nonconf_hist,
                                double* mean_hist, double* scratch, int capacity, fgh_plan ga)
{
    if (!p) return FGH_E_INVALID;
    if (!res_hist && !energy_hist && !nonconf_hist && !mean_hist) {
        if (ga) return FGH_E_INVALID;
        p->hist_res = p->hist_en = p->hist_nc = p->hist_mean = p->hist_scratch = nullptr;
        p->hist_cap = 0;
        p->hist_ga = nullptr;
        return FGH_OK;
    }
    if (capacity < 1) return FGH_E_INVALID;
    if ((nonconf_hist || mean_hist) && !scratch) return FGH_E_INVALID;
    if (p->prec != FGH_FP64) return FGH_E_UNSUPPORTED;
    if (ga) {
        if (!energy_hist || p->rule != FGH_GANI || ga->rule != FGH_GA || ga->d != p->d) return FGH_E_INVALID;
        for (int a = 0; a < p->d; a++)
            if (ga->N[a] != p->N[a]) return FGH_E_INVALID;
    }
    p->hist_res = res_hist;
    p->hist_en = energy_hist;
    p->hist_nc = nonconf_hist;
    p->hist_mean = mean_hist;
    p->hist_scratch = scratch;
    p->hist_cap = capacity;
    p->hist_ga = ga;
    return FGH_OK;
}

fgh_status fgh_gani_bound(fgh_plan gani, fgh_plan ga, const double* E, const double* e, double* bound)
{
    if (!gani || !ga || !E || !e || !bound) return FGH_E_INVALID;
    if (gani->rule != FGH_GANI || ga->rule != FGH_GA || gani->d != ga->d) return FGH_E_INVALID;
    for (int a = 0; a < gani->d; a++)
        if (gani->N[a] != ga->N[a]) return FGH_E_INVALID;
    for (int c = 0; c < gani->d; c++)
        if (!std::isfinite(E[c])) return FGH_E_INVALID;
    // e may still be in flight on the GaNi plan's stream; the work below runs on the Ga plan's.
    HIPOK(hipStreamSynchronize(gani->stream));
    OpPlan opn = gani->op64;
    opn.stream = ga->stream;
    opn.prof = nullptr;
    OpPlan opm = ga->op64;
    opm.prof = nullptr;
    double* y = ga->q64;  // R e on the double grid
    HIPOK(run_prolong(opn, opm, e, y));
    return fgh_effective(ga, E, 1, y, bound, nullptr);
}

/* Adaptive spectral bounds (an extension; the paper's solvers use the pointwise bounds of eq:A):
 * Ritz values of C on the Krylov space of the load
 * from the coefficients of plain CG (Algorithm 2), which are those of the Lanczos process. */
fgh_status fgh_estimate_bounds(fgh_plan p, const double* E, int iters, double* e, double* tri, int* steps,
                               double* lo, double* hi)
{
    if (!p || !E || !e || !lo || !hi || iters < 1 || iters > kMaxLanczos) return FGH_E_INVALID;
    for (int c = 0; c < p->d; c++)
        if (!std::isfinite(E[c])) return FGH_E_INVALID;
    const OpPlan& op = p->op64;
    const long long n = (long long)p->d * p->g.npts;
    const double S = (double)p->g.npts;
    double bb = 0.0, ae2 = 0.0;
    fgh_status s;
    if ((s = rhs<double>(p, E, p->r64, &bb, &ae2))) return s;
    if (!(std::sqrt(bb / S) > kZeroRhs * std::sqrt(ae2 / S))) return FGH_E_INVALID;  // b = 0: no Krylov space
    HIPOK(run_fill<double>(p->stream, n, e, 0.0));
    HIPOK(run_copy<double>(p->stream, n, p->p64, p->r64));
    HIPOK(run_init_loop(op, bb, 0.0, 0.0, -1.0, S, 0.0, 0.0, 0.0, iters));
    const Scalars* h = reinterpret_cast<const Scalars*>(p->host_buf);
    std::vector<double> al, be;
    for (int k = 0; k < iters; k++) {
        HIPOK(cg_body<double>(op, n, e, p->r64, p->p64, p->q64, false));
        HIPOK(hipMemcpyAsync(p->host_buf, op.sc, sizeof(Scalars), hipMemcpyDeviceToHost, op.stream));
        HIPOK(hipStreamSynchronize(op.stream));
        if (!(h->alpha > 0.0) || !std::isfinite(h->alpha)) {
            if (k == 0) return FGH_E_NOT_SPD;  // (C b, b) <= 0
            break;                             // breakdown in round-off: keep T_k
        }
        al.push_back(h->alpha);
        // the residual has vanished to round-off: the Krylov space is invariant, T is complete
        if (k == iters - 1 || !std::isfinite(h->beta) || h->rr <= kLanczosInvariant * kLanczosInvariant * bb) break;
        be.push_back(h->beta);
    }
    // T_m of the Lanczos process: T[0][0] = 1/alpha_0, T[k][k] = 1/alpha_k + beta_{k-1}/alpha_{k-1},
    // T[k][k+1] = sqrt(beta_k)/alpha_k
    const int m = (int)al.size();
    std::vector<double> diag(m), off(m > 0 ? m - 1 : 0);
    for (int k = 0; k < m; k++) diag[k] = 1.0 / al[k] + (k ? be[k - 1] / al[k - 1] : 0.0);
    for (int k = 0; k + 1 < m; k++) off[k] = std::sqrt(be[k]) / al[k];
    *lo = tridiag_eigenvalue(diag, off, 0);
    *hi = tridiag_eigenvalue(diag, off, m - 1);
    if (steps) *steps = m;
    if (tri) {
        for (int k = 0; k < iters; k++) tri[k] = k < m ? diag[k] : 0.0;
        for (int k = 0; k < iters; k++) tri[iters + k] = k + 1 < m ? off[k] : 0.0;
    }
    return FGH_OK;
}

fgh_status fgh_plan_set_bounds(fgh_plan p, double c_A, double C_A)
{
    if (!p || !(c_A > 0.0) || !(C_A >= c_A) || !std::isfinite(C_A)) return FGH_E_INVALID;
    HIPOK(hipStreamSynchronize(p->stream));
    p->cA = c_A;
    p->CA = C_A;
    // the per-phase (A + w I)^{-1} of Eyre-Milton depends on w = sqrt(c_A C_A)
    const double omega = std::sqrt(c_A * C_A);
    for (int i = 0; i < p->nphase; i++) {
        host_shift_inverse(p->d, p->tab[i], omega, p->op64.A.tab_inv[i]);
        host_shift_inverse(p->d, p->tab[i], omega, p->op32.A.tab_inv[i]);
    }
    drop_graph(p);
    return FGH_OK;
}

}  // extern "C"
