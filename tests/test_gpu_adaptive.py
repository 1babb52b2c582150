"""GPU parity of the adaptive spectral bounds (the outlook of Sec. 5): Lanczos estimates of the
spectrum of C = G A from the CG coefficients, and solvers run with bounds set from them.

* Ritz values: the eigenvalues of the tridiagonal T_m that fgh_estimate_bounds builds from its
  CG coefficients match the oracle's Rayleigh-Ritz values on the same Krylov space (explicit
  orthonormal basis, no CG) to 1e-9 of C_A; the host bisection's extremes match numpy's
  eigenvalues of the same T_m to 1e-12; the CG iterate matches the oracle's CG after m steps.
* Closed form: a laminate loaded across its layers has a one-dimensional Krylov space with the
  single Ritz value (a_1 n_0 + a_0 n_1) / n; loaded along them the right-hand side is zero.
* Full size (135^3 spheres): extremes inside [c_A, C_A], Cauchy interlacing of nested T_m,
  determinism of T, the iterate equal to fgh_solve_fixed's CG.
* Solvers with set bounds: Richardson, Chebyshev and Eyre-Milton match the oracle run with the
  same bounds (equal iteration counts, fields to 1e-9); at 45^3 anisotropic, Chebyshev with
  estimated bounds needs far fewer iterations than with the pointwise bounds, same A_H.
"""
import numpy as np
import pytest

from oracle import orc
from paper_1508_02045_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_02045_amd import fgh
    fgh.lib()


def F():
    from paper_1508_02045_amd import fgh as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_plan(N, A_full=None, phase=None, tables=None, kind="phase", rule=0):
    m = F()
    d = len(N)
    if kind == "phase":
        tab = np.stack([I.sym_pack(t[None])[:, 0] for t in tables])
        return m.Plan(N, rule=rule, phase=dev(phase), phase_table=tab.reshape(-1, 3 if d == 2 else 6))
    if kind == "iso":
        return m.Plan(N, rule=rule, A=dev(A_full[..., 0, 0].copy()), a_kind=m.FGH_A_ISO)
    return m.Plan(N, rule=rule, A=dev(I.sym_pack(A_full)), a_kind=m.FGH_A_SYM)


def tri_eigs(est):
    m = est["steps"]
    T = np.diag(est["diag"])
    if m > 1:
        T += np.diag(est["off"], 1) + np.diag(est["off"], -1)
    return np.linalg.eigvalsh(T)


def _case(name):
    rng = np.random.default_rng(7)
    if name == "square63":
        w = I.config1()
        return w.N, w.full(), dict(phase=w.phase, tables=w.tables, kind="phase"), orc.GANI
    if name == "spheres15":
        N = (15, 15, 15)
        ph, _, _ = I.boolean_spheres(N, 2.5, 0.3, rng)
        tables = I.iso_tables(3, [1.0, 100.0])
        return N, I.phase_to_full(ph, tables), dict(phase=ph, tables=tables, kind="phase"), orc.GANI
    if name == "aniso795":
        N = (7, 9, 5)
        A = I.anisotropic_field(N, rng, 1.0, 1e2)
        return N, A, dict(A_full=A, kind="sym"), orc.GANI
    if name == "ga2125":
        N = (21, 25)
        ph = (rng.uniform(size=N) < 0.35).astype(np.uint8)
        A = I.phase_to_full(ph, I.iso_tables(2, [1.0, 30.0]))
        return N, A, dict(A_full=A, kind="iso", rule=1), orc.GA
    raise KeyError(name)


@pytest.mark.parametrize("name", ["square63", "spheres15", "aniso795", "ga2125"])
@pytest.mark.parametrize("m", [1, 4, 12])
def test_ritz_values_match_oracle(name, m):
    N, A, kw, rule = _case(name)
    d = len(N)
    plan = make_plan(N, **kw)
    E = np.array([1.0, -0.5, 0.25][:d])
    print(f"estimate_bounds {name} m={m}", flush=True)
    est = plan.estimate_bounds(E, m)
    assert est["steps"] == m
    ritz = tri_eigs(est)
    AO = A if rule == orc.GANI else orc.ga_assemble(N, A)
    ref = orc.ritz_values(N, rule, AO, E, m)
    _, CA = plan.bounds()
    np.testing.assert_allclose(ritz, ref, rtol=0, atol=1e-9 * CA)
    assert abs(est["lo"] - ritz[0]) <= 1e-12 * CA and abs(est["hi"] - ritz[-1]) <= 1e-12 * CA
    cA, _ = plan.bounds()
    assert cA * (1 - 1e-12) <= est["lo"] <= est["hi"] <= CA * (1 + 1e-12)
    # the iterate is that of m CG steps
    cA, CA = plan.bounds()
    ro = orc.solve(N, rule, AO, E, "cg", cA, CA, 1e-30, fixed_iters=m)
    eg = est["e"].cpu().numpy()
    scale = np.linalg.norm(ro.e + E.reshape((d,) + (1,) * d))
    assert np.linalg.norm(eg - ro.e) / scale <= 1e-9


@pytest.mark.parametrize("N", [(21, 15, 9), (9, 35)])
def test_laminate_one_step(N):
    m = F()
    d = len(N)
    rng = np.random.default_rng(len(N))
    lp = (rng.uniform(size=N[0]) < 0.4).astype(np.uint8)
    lp[0], lp[1] = 1, 0
    a0, a1 = 1.0, 25.0
    ph = I.laminate(N, 0, lp)
    plan = make_plan(N, phase=ph, tables=I.iso_tables(d, [a0, a1]), kind="phase")
    E = np.zeros(d)
    E[0] = 1.0
    print(f"estimate_bounds laminate {N}", flush=True)
    est = plan.estimate_bounds(E, 10)
    n1, n = int(lp.sum()), N[0]
    lam = (a1 * (n - n1) + a0 * n1) / n
    assert est["steps"] == 1
    assert abs(est["lo"] - lam) <= 1e-12 * a1 and abs(est["hi"] - lam) <= 1e-12 * a1
    E = np.zeros(d)
    E[1] = 1.0
    with pytest.raises(m.FghError) as ex:
        plan.estimate_bounds(E, 10)
    assert ex.value.status == m.FGH_E_INVALID


def test_invalid_arguments():
    m = F()
    w = I.config1()
    plan = make_plan(w.N, phase=w.phase, tables=w.tables, kind="phase")
    for iters in (0, 5000):
        with pytest.raises(m.FghError):
            plan.estimate_bounds(w.E, iters)
    for cA, CA in ((0.0, 1.0), (2.0, 1.0), (1.0, float("inf")), (-1.0, 3.0)):
        with pytest.raises(m.FghError):
            plan.set_bounds(cA, CA)
    assert plan.bounds() == (1.0, 10.0)


def test_full_size_spheres135():
    """The 135^3 Boolean-spheres workload: properties that hold at any size."""
    m = F()
    w = I.config2()
    tab = np.stack([I.sym_pack(t[None])[:, 0] for t in w.tables])
    plan = m.Plan(w.N, phase=dev(w.phase), phase_table=tab)
    cA, CA = plan.bounds()
    print("estimate_bounds 135^3 m=30", flush=True)
    est = plan.estimate_bounds(w.E, 30)
    assert est["steps"] == 30
    assert cA * (1 - 1e-12) <= est["lo"] < est["hi"] <= CA * (1 + 1e-12)
    T = np.diag(est["diag"]) + np.diag(est["off"], 1) + np.diag(est["off"], -1)
    lo_prev, hi_prev = np.inf, -np.inf
    for k in range(1, 31):
        ev = np.linalg.eigvalsh(T[:k, :k])
        assert ev[0] <= lo_prev + 1e-12 * CA and ev[-1] >= hi_prev - 1e-12 * CA
        lo_prev, hi_prev = ev[0], ev[-1]
    assert abs(est["lo"] - lo_prev) <= 1e-12 * CA and abs(est["hi"] - hi_prev) <= 1e-12 * CA
    # deterministic: a shorter run builds the leading block exactly
    est12 = plan.estimate_bounds(w.E, 12)
    assert np.array_equal(est12["diag"], est["diag"][:12]) and np.array_equal(est12["off"], est["off"][:11])
    # the iterate is fgh_solve_fixed's CG iterate after the same number of bodies
    e, st, _ = plan.solve_fixed("cg", w.E, 30)
    assert st == 0
    a, b = est["e"].cpu().numpy(), e.cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)


@pytest.mark.parametrize("solver", ["richardson", "chebyshev"])
def test_solvers_with_set_bounds_match_oracle_sym(solver):
    N = (15, 15, 15)
    A = I.anisotropic_field(N, np.random.default_rng(5))
    plan = make_plan(N, A_full=A, kind="sym")
    E = np.array([1.0, 0.0, 0.0])
    est = plan.estimate_bounds(E, 30)
    c, C = 0.9 * est["lo"], 1.02 * est["hi"]
    plan.set_bounds(c, C)
    assert plan.bounds() == (c, C)
    tol = 1e-8
    print(f"adaptive {solver} 15^3 [{c:.4g}, {C:.4g}]", flush=True)
    e, st, stats = plan.solve(solver, E, tol, max_iter=5000)
    assert st == 0, stats
    r = orc.solve(N, orc.GANI, A, E, solver, c, C, tol, max_iter=5000)
    assert r.status == 0
    m_o = len(r.res_hist) - 1
    assert abs(stats[0]["iters"] - m_o) <= 1 and (stats[0]["iters"] == m_o or
                                                   abs(r.res_hist[min(stats[0]["iters"], m_o)] - tol) <= 1e-6 * tol)
    ro = orc.solve(N, orc.GANI, A, E, solver, c, C, tol, fixed_iters=stats[0]["iters"])
    scale = np.linalg.norm(ro.e + E.reshape(3, 1, 1, 1))
    assert np.linalg.norm(e.cpu().numpy() - ro.e) / scale <= 1e-9


def test_eyre_milton_with_set_bounds_matches_oracle_phase():
    """Phase plans keep (A + w I)^{-1} per phase; set_bounds must rebuild it for the new w."""
    w = I.config1()
    A = w.full()
    plan = make_plan(w.N, phase=w.phase, tables=w.tables, kind="phase")
    e0, st0, s0 = plan.solve("eyre_milton", w.E, 1e-8)
    c, C = 1.4, 7.5
    plan.set_bounds(c, C)
    print("adaptive eyre_milton 63^2", flush=True)
    e, st, stats = plan.solve("eyre_milton", w.E, 1e-8, max_iter=5000)
    assert st == 0 and st0 == 0
    r = orc.solve(w.N, orc.GANI, A, w.E, "eyre_milton", c, C, 1e-8, max_iter=5000)
    m_o = len(r.res_hist) - 1
    assert stats[0]["iters"] == m_o or abs(stats[0]["iters"] - m_o) <= 1
    ro = orc.solve(w.N, orc.GANI, A, w.E, "eyre_milton", c, C, 1e-8, fixed_iters=stats[0]["iters"])
    scale = np.linalg.norm(ro.e + w.E[:, None, None])
    assert np.linalg.norm(e.cpu().numpy() - ro.e) / scale <= 1e-9


def test_estimated_bounds_speed_up_chebyshev_aniso45():
    """45^3 per-voxel anisotropic field (eigenvalues log-uniform in [1, 1e3]): the spectrum of C
    is much narrower than the pointwise [c_A, C_A], so Chebyshev on estimated bounds takes far
    fewer iterations and reaches the same A_H."""
    w = I.config3(45)
    plan = make_plan(w.N, A_full=w.A_full, kind="sym")
    E = w.E
    tol = 1e-10
    print("chebyshev 45^3 default bounds", flush=True)
    e_cg, st, s_cg = plan.solve("cg", E, tol, max_iter=20000)
    assert st == 0
    e_d, st, s_d = plan.solve("chebyshev", E, tol, max_iter=20000)
    assert st == 0
    est = plan.estimate_bounds(E, 40)
    plan.set_bounds(0.9 * est["lo"], 1.02 * est["hi"])
    print(f"chebyshev 45^3 estimated bounds [{est['lo']:.4g}, {est['hi']:.4g}]", flush=True)
    e_a, st, s_a = plan.solve("chebyshev", E, tol, max_iter=20000)
    assert st == 0
    assert s_a[0]["iters"] <= 0.6 * s_d[0]["iters"], (s_a[0]["iters"], s_d[0]["iters"])
    en = [plan.effective(E, x)[0][0, 0] for x in (e_cg, e_d, e_a)]
    assert abs(en[2] - en[0]) <= 1e-9 * en[0] and abs(en[1] - en[0]) <= 1e-9 * en[0]
