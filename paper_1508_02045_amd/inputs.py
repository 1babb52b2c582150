"""Seeded synthetic microstructures and workload configurations.

This module generates inputs only: phase maps, per-voxel coefficient fields and loads.  It
holds none of the homogenization arithmetic, so both the GPU path and the oracle can be fed
the very same bytes from it.

Grid convention (paper Sec. 2.1): axis alpha has an odd number n of points; array index i
stands for the signed index m = i if 2 i < n else i - n, i.e. the grid point x = m / n of the
unit cell (-1/2, 1/2)^d.  A "centred" inclusion is therefore centred at the origin, which sits
at array index 0 and wraps around the array ends.

The paper's own workloads are a 36 % square inclusion (85 x 85, contrast 100) and a fly-ash
bitmap that is not available; the configurations here are seeded stand-ins with the same
two-phase, pixel-wise constant, high-contrast structure (Sec. 4, cell types).
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Optional, Sequence, Tuple

import numpy as np

ROOT_SEED = 1508


def config_rng(i: int) -> np.random.Generator:
    """PCG64 generator of workload configuration i (0-based)."""
    return np.random.default_rng(np.random.SeedSequence(ROOT_SEED).spawn(5)[i])


def signed_indices(n: int) -> np.ndarray:
    i = np.arange(n)
    return np.where(2 * i < n, i, i - n)


def _mesh(N: Sequence[int]):
    return np.meshgrid(*[signed_indices(n) for n in N], indexing="ij")


def centred_box(N: Sequence[int], half: Sequence[int] | int) -> np.ndarray:
    """uint8 phase map: 1 where |m_a| <= half_a on every axis, else 0 (box of 2 half + 1 pixels)."""
    d = len(N)
    if np.isscalar(half):
        half = [int(half)] * d
    inside = np.ones(tuple(N), dtype=bool)
    for m, h in zip(_mesh(N), half):
        inside &= np.abs(m) <= h
    return inside.astype(np.uint8)


def paper_square(N: Sequence[int], side: float = 0.6) -> np.ndarray:
    """The paper's square (cube) inclusion of side `side` centred in the cell: pixel m inside iff
    |m_a / N_a| < side / 2 on every axis (36 % for side 0.6; 51 of 85 or 9 of 15 pixels)."""
    inside = np.ones(tuple(N), dtype=bool)
    for m, n in zip(_mesh(N), N):
        inside &= np.abs(m) * 2 < side * n
    return inside.astype(np.uint8)


def laminate(N: Sequence[int], axis: int, layer_phase: Sequence[int]) -> np.ndarray:
    """Pixel-aligned laminate: the phase depends only on the index along `axis`
    (layer_phase[i] for array index i)."""
    N = tuple(N)
    lp = np.asarray(layer_phase, dtype=np.uint8)
    assert lp.shape == (N[axis],)
    shape = [1] * len(N)
    shape[axis] = N[axis]
    return np.broadcast_to(lp.reshape(shape), N).copy()


def boolean_spheres(N: Sequence[int], radius: float, target_fraction: float,
                    rng: np.random.Generator, max_spheres: int = 100000) -> Tuple[np.ndarray, float, int]:
    """Boolean model of overlapping spheres (discs in 2D).

    Centres are uniform continuous in [0, N_a) (voxel units).  Voxel i is inside a sphere if
    its periodic minimum-image distance to the centre is <= radius.  Spheres are added one at a
    time until the voxel fraction first reaches target_fraction.
    Returns (phase map uint8, achieved fraction, number of spheres)."""
    N = tuple(int(n) for n in N)
    d = len(N)
    phase = np.zeros(N, dtype=bool)
    r = float(radius)
    rad = int(np.ceil(r))
    offs = np.arange(-rad - 1, rad + 2)
    total = float(np.prod(N))
    inside = 0
    count = 0
    for count in range(1, max_spheres + 1):
        c = rng.uniform(0.0, 1.0, size=d) * np.asarray(N, dtype=np.float64)
        # candidate voxels around the centre (periodic wrap)
        base = np.floor(c).astype(np.int64)
        idx = [((base[a] + offs) % N[a]) for a in range(d)]
        dist2 = np.zeros([len(offs)] * d)
        for a in range(d):
            delta = (base[a] + offs).astype(np.float64) - c[a]
            shape = [1] * d
            shape[a] = len(offs)
            dist2 = dist2 + (delta ** 2).reshape(shape)
        mask = dist2 <= r * r
        sub = np.ix_(*idx)
        block = phase[sub]
        phase[sub] = block | mask
        if len(offs) <= min(N):
            inside += int(np.count_nonzero(mask & ~block))
        else:  # the candidate block wraps onto itself: recount
            inside = int(np.count_nonzero(phase))
        if inside / total >= target_fraction:
            break
    return phase.astype(np.uint8), float(inside / total), count


def haar_rotations(n: int, d: int, rng: np.random.Generator) -> np.ndarray:
    """n Haar-distributed rotations (QR of a standard normal matrix with the diagonal of R made
    positive, then the determinant fixed to +1)."""
    Z = rng.standard_normal((n, d, d))
    Q, R = np.linalg.qr(Z)
    s = np.sign(np.diagonal(R, axis1=1, axis2=2))
    s[s == 0] = 1.0
    Q = Q * s[:, None, :]
    det = np.linalg.det(Q)
    Q[det < 0, :, 0] *= -1.0
    return Q


def anisotropic_field(N: Sequence[int], rng: np.random.Generator, lam_lo: float = 1.0,
                      lam_hi: float = 1e3) -> np.ndarray:
    """Per-voxel SPD A = R^T diag(lambda) R, R Haar-random, lambda log-uniform in [lam_lo, lam_hi].
    Returns [*N, d, d] float64 (exactly symmetric)."""
    N = tuple(N)
    d = len(N)
    n = int(np.prod(N))
    R = haar_rotations(n, d, rng)
    lam = 10.0 ** rng.uniform(np.log10(lam_lo), np.log10(lam_hi), size=(n, d))
    A = np.einsum("nki,nk,nkj->nij", R, lam, R)
    A = 0.5 * (A + np.transpose(A, (0, 2, 1)))
    return A.reshape(N + (d, d))


def phase_to_full(phase: np.ndarray, tables: Sequence[np.ndarray]) -> np.ndarray:
    """Expand a phase map to a full coefficient field [*grid, d, d]."""
    tables = np.asarray(tables, dtype=np.float64)
    return tables[phase.astype(np.int64)]


def iso_tables(d: int, values: Sequence[float]) -> np.ndarray:
    return np.stack([v * np.eye(d) for v in values])


def sym_pack(A: np.ndarray) -> np.ndarray:
    """[*grid, d, d] symmetric -> [ncoef, *grid] packed upper triangle, row by row
    (2D: a00 a01 a11; 3D: a00 a01 a02 a11 a12 a22)."""
    d = A.shape[-1]
    comps = [A[..., i, j] for i in range(d) for j in range(i, d)]
    return np.ascontiguousarray(np.stack(comps))


def sha256(*arrays: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


@dataclasses.dataclass
class Workload:
    name: str
    N: Tuple[int, ...]
    phase: Optional[np.ndarray]          # uint8 phase map, or None
    tables: Optional[np.ndarray]         # [n_phases, d, d]
    A_full: Optional[np.ndarray]         # [*N, d, d] when not a phase map
    E: np.ndarray
    contrast: float
    fraction: float
    note: str = ""

    @property
    def d(self):
        return len(self.N)

    def full(self) -> np.ndarray:
        if self.A_full is not None:
            return self.A_full
        return phase_to_full(self.phase, self.tables)


def config1() -> Workload:
    """2D, 63 x 63, centred 21 x 21 square (fraction 441/3969), A = I / 10 I, E = (1, 0)."""
    N = (63, 63)
    ph = centred_box(N, 10)
    return Workload("c1_square2d_63", N, ph, iso_tables(2, [1.0, 10.0]), None,
                    np.array([1.0, 0.0]), 10.0, float(ph.mean()))


def config2(N: int = 135, radius: float = 8.0, fraction: float = 0.30, contrast: float = 100.0) -> Workload:
    """3D Boolean spheres r = 8 voxels, volume fraction 0.30, A = I / 100 I, E = e1 at 135^3."""
    ph, frac, ns = boolean_spheres((N, N, N), radius, fraction, config_rng(1))
    return Workload(f"c2_spheres3d_{N}", (N, N, N), ph, iso_tables(3, [1.0, contrast]), None,
                    np.array([1.0, 0.0, 0.0]), contrast, frac, note=f"{ns} spheres")


def config3(N: int = 63) -> Workload:
    """3D per-voxel anisotropic SPD field (Haar rotations, eigenvalues log-uniform in [1, 1e3])."""
    A = anisotropic_field((N, N, N), config_rng(2))
    return Workload(f"c3_aniso3d_{N}", (N, N, N), None, None, A, np.array([1.0, 0.0, 0.0]), 1e3, 0.0)


def config4(contrast: float, N: int = 243, radius: float = 12.0, fraction: float = 0.25) -> Workload:
    """3D Boolean spheres r = 12, fraction 0.25, A = I / rho I, E = e1 at 243^3."""
    ph, frac, ns = boolean_spheres((N, N, N), radius, fraction, config_rng(3))
    return Workload(f"c4_spheres3d_{N}_rho{contrast:g}", (N, N, N), ph, iso_tables(3, [1.0, contrast]),
                    None, np.array([1.0, 0.0, 0.0]), contrast, frac, note=f"{ns} spheres")


def cube_side_for_fraction(n: int, d: int, f: float) -> int:
    """Odd side (pixels) of a centred square/cube whose area fraction is nearest f."""
    best = 1
    for side in range(1, n + 1, 2):
        if abs((side / n) ** d - f) < abs((best / n) ** d - f):
            best = side
    return best


def serving_requests(count: int, rng: np.random.Generator):
    """A seeded stream of homogenization requests of mixed shape (the served workload).

    d uniform in {2, 3}; exact integration (Ga) with probability 0.2 for N in {41, 63};
    otherwise 2D N in {81, 243, 729} or 3D N in {45, 81, 135, 243}.  Microstructure: a centred
    square/cube or a Boolean model of discs/spheres of radius max(2, round(N / 20)), inclusion
    fraction U[0.1, 0.4]; A = I / rho I with rho log-uniform in [10, 1e4]; E = e1; solver CG or
    Eyre-Milton (CG for Ga); tolerance 1e-6 or 1e-8."""
    reqs = []
    for _ in range(count):
        d = int(rng.integers(2, 4))
        ga = rng.uniform() < 0.2
        if ga:
            n = int(rng.choice([41, 63]))
        elif d == 2:
            n = int(rng.choice([81, 243, 729]))
        else:
            n = int(rng.choice([45, 81, 135, 243]))
        N = (n,) * d
        f = float(rng.uniform(0.1, 0.4))
        rho = float(10.0 ** rng.uniform(1.0, 4.0))
        if rng.uniform() < 0.5:
            phase = centred_box(N, cube_side_for_fraction(n, d, f) // 2)
            micro = "box"
        else:
            phase, f, _ = boolean_spheres(N, max(2, round(n / 20)), f, rng)
            micro = "spheres"
        solver = "cg" if ga or rng.uniform() < 0.5 else "eyre_milton"
        tol = float(rng.choice([1e-6, 1e-8]))
        E = np.zeros(d)
        E[0] = 1.0
        reqs.append({"d": d, "N": N, "rule": 1 if ga else 0, "phase": phase, "tables": iso_tables(d, [1.0, rho]),
                     "rho": rho, "fraction": float(phase.mean()), "micro": micro, "solver": solver, "tol": tol,
                     "E": E})
    return reqs
