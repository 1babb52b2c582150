"""FFT-free dense Galerkin brute force (test helper, numpy only).

Trial/test functions are the gradient modes psi_k(x) = k exp(2 pi i k.x), k in Z_N \\ {0}
(paper Sec. 2: the admissible space is curl-free, zero-mean trigonometric polynomials).

GaNi (eq:GaNi): the bilinear form is the trapezoidal sum over the N grid, so the Galerkin
matrix is assembled from the fields psi_k sampled at the grid points.
Ga (eq:Ga, eq:Ga_eval): the bilinear form is the exact integral; for a pixel-wise constant A
it is  a(psi_k, psi_l) = l^T A^(l - k) k  with A^(n) the exact Fourier coefficient of A,
which is computed here by integrating exp(-2 pi i n x) over each pixel in closed form.
No DFT, no double grid, no projection: an independent route to A_H and to the fields.
"""
import itertools

import numpy as np


def freqs(N):
    rng = [np.arange(-(n // 2), n // 2 + 1) for n in N]
    K = np.array(list(itertools.product(*rng)), dtype=np.int64)
    return K[np.any(K != 0, axis=1)]


def grid_points(n_grid):
    axes = []
    for n in n_grid:
        i = np.arange(n)
        axes.append(np.where(2 * i < n, i, i - n) / n)
    P = np.array(list(itertools.product(*axes)))
    return P


def _modes_at(K, P):
    """Matrix Phi [(d * npts), nk]: column k is psi_k at the points P, component-major."""
    d = K.shape[1]
    ph = np.exp(2j * np.pi * (P @ K.T))  # [npts, nk]
    cols = [ph * K[None, :, a] for a in range(d)]  # each [npts, nk]
    return np.concatenate(cols, axis=0)


def gani_solve(N, A_full, E):
    """Returns (e field [d, *N], energy) for GaNi."""
    N = tuple(N)
    d = len(N)
    K = freqs(N)
    P = grid_points(N)
    npts = P.shape[0]
    Phi = _modes_at(K, P)
    A = A_full.reshape(npts, d, d)
    # W Phi: pointwise A times the field
    Phi_c = Phi.reshape(d, npts, -1)
    WPhi = np.einsum("pab,bpk->apk", A, Phi_c).reshape(d * npts, -1)
    Kmat = Phi.conj().T @ WPhi / npts
    AE = np.einsum("pab,b->ap", A, E).reshape(-1)
    f = -(Phi.conj().T @ AE) / npts
    c = np.linalg.solve(Kmat, f)
    e = (Phi @ c).real.reshape((d,) + N)
    u = e.reshape(d, npts) + E[:, None]
    en = np.einsum("ap,pab,bp->", u, A, u) / npts
    return e, en


def pixel_fourier_coeffs(N, A_full, nvecs):
    """Exact A^(n) = int A(x) exp(-2 pi i n.x) dx for pixel-wise constant A (pixel m centred at
    m/N, width 1/N).  Returns [len(nvecs), d, d] complex."""
    N = tuple(N)
    d = len(N)
    out = np.zeros((len(nvecs), d, d), dtype=np.complex128)
    per_axis = []
    for a, n in enumerate(N):
        i = np.arange(n)
        xm = np.where(2 * i < n, i, i - n) / n
        h = 1.0 / n
        nn = nvecs[:, a][:, None].astype(np.float64)
        lo, hi = xm[None, :] - h / 2, xm[None, :] + h / 2
        with np.errstate(divide="ignore", invalid="ignore"):
            val = (np.exp(-2j * np.pi * nn * hi) - np.exp(-2j * np.pi * nn * lo)) / (-2j * np.pi * nn)
        val = np.where(nn == 0, h, val)
        per_axis.append(val)  # [nvec, n]
    # contract A over the grid: sum_m A_m prod_a I_a(n_a, m_a)
    Ar = A_full.reshape(N + (d * d,))
    if d == 2:
        out = np.einsum("vi,vj,ijc->vc", per_axis[0], per_axis[1], Ar)
    else:
        out = np.einsum("vi,vj,vk,ijkc->vc", per_axis[0], per_axis[1], per_axis[2], Ar)
    return out.reshape(len(nvecs), d, d)


def ga_solve(N, A_full, E):
    """Returns (e field on the double grid [d, *(2N-1)], energy) for Ga."""
    N = tuple(N)
    d = len(N)
    K = freqs(N)
    nk = K.shape[0]
    diffs = (K[:, None, :] - K[None, :, :]).reshape(-1, d)  # l - k for (l, k)
    Ahat_diff = pixel_fourier_coeffs(N, A_full, diffs).reshape(nk, nk, d, d)
    Kmat = np.einsum("la,lkab,kb->lk", K, Ahat_diff, K)
    Ahat_l = pixel_fourier_coeffs(N, A_full, K)
    f = -np.einsum("la,lab,b->l", K, Ahat_l, E)
    c = np.linalg.solve(Kmat, f)
    A0 = pixel_fourier_coeffs(N, A_full, np.zeros((1, d), dtype=np.int64))[0].real
    en = float(E @ A0 @ E - (c.conj() @ f).real)
    M = tuple(2 * n - 1 for n in N)
    P = grid_points(M)
    e = (_modes_at(K, P) @ c).real.reshape((d,) + M)
    return e, en


def gani_matrices(N, A_full, E):
    """GaNi Galerkin matrices in the gradient-mode basis: stiffness K (from A), mass M (the
    grid inner product of the modes) and load f = -(A E, psi_l).  The eigenvalues of K c = lam M c
    are those of C = G A on compatible fields."""
    N = tuple(N)
    d = len(N)
    K = freqs(N)
    P = grid_points(N)
    npts = P.shape[0]
    Phi = _modes_at(K, P)
    A = A_full.reshape(npts, d, d)
    Phi_c = Phi.reshape(d, npts, -1)
    WPhi = np.einsum("pab,bpk->apk", A, Phi_c).reshape(d * npts, -1)
    Kmat = Phi.conj().T @ WPhi / npts
    Mmat = Phi.conj().T @ Phi / npts
    AE = np.einsum("pab,b->ap", A, E).reshape(-1)
    f = -(Phi.conj().T @ AE) / npts
    return Kmat, Mmat, f


def ga_matrices(N, A_full, E):
    """Ga Galerkin matrices (exact integrals): K from the exact Fourier coefficients of the
    pixel-wise constant A, M = diag(|k|^2) (the modes are orthogonal in L2), f = -(A E, psi_l)."""
    N = tuple(N)
    d = len(N)
    K = freqs(N)
    nk = K.shape[0]
    diffs = (K[:, None, :] - K[None, :, :]).reshape(-1, d)
    Ahat_diff = pixel_fourier_coeffs(N, A_full, diffs).reshape(nk, nk, d, d)
    Kmat = np.einsum("la,lkab,kb->lk", K, Ahat_diff, K)
    Mmat = np.diag(np.sum(K * K, axis=1).astype(np.float64)).astype(np.complex128)
    Ahat_l = pixel_fourier_coeffs(N, A_full, K)
    f = -np.einsum("la,lab,b->l", K, Ahat_l, E)
    return Kmat, Mmat, f
