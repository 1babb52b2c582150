"""ctypes wrapper of the FP64 oracle (fgh_oracle.c).

TEST INFRASTRUCTURE ONLY.  Arrays are numpy float64, C-contiguous:
  vector field  [d, *grid]        coefficient field  [*grid, d, d]
GaNi works on the N grid, Ga on the double grid M = 2N - 1 (paper Sec. 2.2-2.3).
"""
import ctypes
import numpy as np

from . import build as _build

GANI, GA = 0, 1
RICHARDSON, CG, CHEBYSHEV, EYRE_MILTON = 0, 1, 2, 3
SOLVER_NAMES = {"richardson": RICHARDSON, "cg": CG, "chebyshev": CHEBYSHEV, "eyre_milton": EYRE_MILTON}
OK, E_INVALID, E_NO_CONVERGENCE, E_DIVERGED = 0, 1, 5, 6

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        L.orc_dft.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_int]
        L.orc_apply_at.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_int, _ip, _dp]
        L.orc_apply.argtypes = [ctypes.c_int, _ip, ctypes.c_int, _dp, _dp, _dp]
        L.orc_project.argtypes = [ctypes.c_int, _ip, ctypes.c_int, _dp, _dp]
        L.orc_ga_assemble.argtypes = [ctypes.c_int, _ip, _dp, _dp]
        L.orc_prolong.argtypes = [ctypes.c_int, _ip, _dp, _dp]
        L.orc_spectral_bounds.argtypes = [ctypes.c_int, ctypes.c_long, _dp, _dp, _dp]
        L.orc_bilinear.argtypes = [ctypes.c_int, _ip, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_flux.argtypes = [ctypes.c_int, _ip, ctypes.c_int, _dp, _dp, _dp, _dp]
        L.orc_solve.argtypes = [ctypes.c_int, _ip, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, _dp, _ip, _dp, _dp, _dp]
        L.orc_num_threads.argtypes = []
        for f in (L.orc_dft, L.orc_apply_at, L.orc_apply, L.orc_project, L.orc_ga_assemble, L.orc_prolong,
                  L.orc_spectral_bounds, L.orc_bilinear, L.orc_flux, L.orc_solve, L.orc_num_threads):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _ints(v):
    arr = (ctypes.c_int * len(v))(*[int(t) for t in v])
    return arr


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def double_grid(N):
    return tuple(2 * int(n) - 1 for n in N)


def op_grid(N, rule):
    return tuple(int(n) for n in N) if rule == GANI else double_grid(N)


def num_threads():
    return lib().orc_num_threads()


def dft(c, inverse=False):
    """Naive separable DFT of a complex grid (forward carries 1/|grid|; eq:DFT)."""
    c = np.asarray(c, dtype=np.complex128)
    re = _f64(c.real.copy())
    im = _f64(c.imag.copy())
    st = lib().orc_dft(c.ndim, _ints(c.shape), _d(re), _d(im), 1 if inverse else 0)
    assert st == OK, st
    return re + 1j * im


def apply_at(N, A, x, ks):
    """Fourier coefficients G(k) (A x)^(k) of the GaNi operator at the listed signed frequencies
    ks [nk][d], by direct sums over the grid (no transform); [nk][d] complex."""
    d = len(N)
    A = _f64(A)
    x = _f64(x)
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int32).reshape(-1, d))
    out = np.empty((ks.shape[0], d, 2), dtype=np.float64)
    st = lib().orc_apply_at(d, _ints(N), _d(A), _d(x), ks.shape[0], ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                            _d(out))
    assert st == OK, st
    return out[..., 0] + 1j * out[..., 1]


def apply(N, rule, A, x):
    """y = C x = G A x on the integration grid (eq:linsys)."""
    d = len(N)
    A = _f64(A)
    x = _f64(x)
    y = np.empty_like(x)
    st = lib().orc_apply(d, _ints(N), rule, _d(A), _d(x), _d(y))
    assert st == OK, st
    return y


def project(N, rule, x):
    d = len(N)
    x = _f64(x)
    y = np.empty_like(x)
    st = lib().orc_project(d, _ints(N), rule, _d(x), _d(y))
    assert st == OK, st
    return y


def ga_assemble(N, A_N):
    """A on the N grid [*N, d, d] -> A_{2N-1} on the double grid (eq:Ga_exact_integration)."""
    d = len(N)
    A_N = _f64(A_N)
    out = np.empty(double_grid(N) + (d, d), dtype=np.float64)
    st = lib().orc_ga_assemble(d, _ints(N), _d(A_N), _d(out))
    assert st == OK, st
    return out


def prolong(N, uN):
    """R_{N,2N-1}: trigonometric interpolation from the N grid to the double grid."""
    d = len(N)
    uN = _f64(uN)
    out = np.empty((d,) + double_grid(N), dtype=np.float64)
    st = lib().orc_prolong(d, _ints(N), _d(uN), _d(out))
    assert st == OK, st
    return out


def spectral_bounds(A):
    d = A.shape[-1]
    A = _f64(A)
    npts = A.size // (d * d)
    lo = ctypes.c_double()
    hi = ctypes.c_double()
    lib().orc_spectral_bounds(d, npts, _d(A), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def bilinear(N, rule, A, Ei, ei, Ej, ej):
    """(A (E_i + e_i), E_j + e_j)_2 on the integration grid (eq:ev_bounds)."""
    d = len(N)
    A = _f64(A)
    Ei = _f64(Ei)
    Ej = _f64(Ej)
    ei_c = _f64(ei) if ei is not None else None
    ej_c = _f64(ej) if ej is not None else None
    out = ctypes.c_double()
    st = lib().orc_bilinear(d, _ints(N), rule, _d(A), _d(Ei), _d(ei_c) if ei_c is not None else None,
                            _d(Ej), _d(ej_c) if ej_c is not None else None, ctypes.byref(out))
    assert st == OK, st
    return out.value


def flux(N, rule, A, E, e):
    d = len(N)
    A = _f64(A)
    E = _f64(E)
    e_c = _f64(e) if e is not None else None
    out = np.empty(d, dtype=np.float64)
    st = lib().orc_flux(d, _ints(N), rule, _d(A), _d(E), _d(e_c) if e_c is not None else None, _d(out))
    assert st == OK, st
    return out


class SolveResult:
    def __init__(self, e, iters, status, res_hist, energy_hist, rel_res_true):
        self.e = e
        self.iters = iters
        self.status = status
        self.res_hist = res_hist
        self.energy_hist = energy_hist
        self.rel_res_true = rel_res_true


def solve(N, rule, A, E, solver, cA, CA, tol, max_iter=10000, fixed_iters=0, energy=False):
    """Run Alg. 1-4 step by step (see fgh_oracle.c for the exact conventions)."""
    d = len(N)
    if isinstance(solver, str):
        solver = SOLVER_NAMES[solver]
    A = _f64(A)
    E = _f64(E)
    g = op_grid(N, rule)
    e = np.empty((d,) + g, dtype=np.float64)
    cap = fixed_iters if fixed_iters > 0 else max_iter
    res = np.zeros(cap + 1, dtype=np.float64)
    en = np.zeros(cap + 1, dtype=np.float64) if energy else None
    iters = ctypes.c_int()
    rt = ctypes.c_double()
    st = lib().orc_solve(d, _ints(N), rule, _d(A), _d(E), solver, float(cA), float(CA), float(tol),
                         int(max_iter), int(fixed_iters), _d(e), ctypes.byref(iters), _d(res),
                         _d(en) if en is not None else None, ctypes.byref(rt))
    m = iters.value
    return SolveResult(e, m, st, res[: m + 1].copy(), en[: m + 1].copy() if en is not None else None, rt.value)


def effective_tensor(N, rule, A, fields):
    """A_H[i][j] = (A(e_j + e^(j)), e_i + e^(i))_2 from the d unit-load solutions (eq:ev_bounds)."""
    d = len(N)
    I = np.eye(d)
    AH = np.empty((d, d))
    for i in range(d):
        for j in range(d):
            AH[i, j] = bilinear(N, rule, A, I[j], fields[j], I[i], fields[i])
    return AH


def energy(N, rule, A, E, e):
    return bilinear(N, rule, A, E, e, E, e)


def krylov_rhs(N, rule, A, E):
    """b = -C E, the right-hand side of the fluctuation system C e = b (eq:linsys), with E the
    constant field on the integration grid."""
    d = len(N)
    g = op_grid(N, rule)
    Ef = np.empty((d,) + g, dtype=np.float64)
    for a in range(d):
        Ef[a] = E[a]
    return -apply(N, rule, A, Ef)


def ritz_values(N, rule, A, E, m, breakdown=1e-10):
    """Ritz values of C = G A on the Krylov space K_m(C, b), b = -C E.

    This is the plain Rayleigh-Ritz definition behind the library's adaptive bounds (an extension:
    the paper's solvers take the pointwise bounds of eq:A): an orthonormal basis Q of span{b, C b, ..., C^(m-1) b} is built by
    Gram-Schmidt, applied twice to each new vector, and the eigenvalues of the m x m matrix
    Q^T C Q are returned in ascending order.  The inner product is the plain sum over the grid
    and the components.  When C^j b already lies in the span of the earlier vectors (relative
    norm below `breakdown`) the space is invariant and fewer than m values are returned; a zero
    b (round-off compared with A E) gives none.  Near the dimension of the invariant space the
    basis is only as good as round-off lets it be, so use m well below it.
    Test infrastructure: the GPU path builds the same values from its CG coefficients instead."""
    b = krylov_rhs(N, rule, A, E).reshape(-1)
    nb = np.linalg.norm(b)
    # b that is round-off next to A E (e.g. a laminate loaded along its layers) spans nothing
    AE = np.einsum("...ab,b->...a", _f64(A), _f64(E))
    if not nb > 1e-12 * np.sqrt(np.sum(AE * AE)):
        return np.zeros(0)
    shape = b.shape
    Q = [b / nb]
    CQ = []
    field_shape = (len(N),) + op_grid(N, rule)
    for j in range(m):
        w = apply(N, rule, A, Q[j].reshape(field_shape)).reshape(shape)
        CQ.append(w)
        if j == m - 1:
            break
        v = w.copy()
        for _ in range(2):
            for q in Q:
                v = v - (q @ v) * q
        nv = np.linalg.norm(v)
        if nv <= breakdown * np.linalg.norm(w):
            break
        Q.append(v / nv)
    Qm = np.stack(Q[: len(CQ)], axis=1)
    T = Qm.T @ np.stack(CQ, axis=1)
    T = 0.5 * (T + T.T)
    return np.linalg.eigvalsh(T)
