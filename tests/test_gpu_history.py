"""GPU parity of the per-iteration histories (Sec. 4.2 residuals; Sec. 4.3 eq:guar_upper_bound_m
energies and the GaNi guaranteed-bound monitor) against the oracle, entry by entry.

Tolerances: energies 1e-10 relative (as A_H); the residual quantity 1e-4 relative plus 1e-11
absolute, since late entries are ratios of norms near tol * ||b|| whose round-off, accumulated
over the iterations, is about 1e-13 ||b||."""
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


def plan(N, A, rule=0, precision=0):
    m = F()
    return m.Plan(N, rule=rule, precision=precision, A=dev(I.sym_pack(A)), a_kind=m.FGH_A_SYM, c_A=1.0,
                  C_A=float(np.linalg.eigvalsh(A).max()))


def check_res(gpu, ref):
    assert np.all(np.abs(gpu - ref) <= 1e-4 * np.abs(ref) + 1e-11), (gpu, ref)


def check_en(gpu, ref):
    assert np.all(np.abs(gpu - ref) <= 1e-10 * np.abs(ref)), np.max(np.abs(gpu - ref) / np.abs(ref))


CASES = [((15, 21), 0, "richardson"), ((15, 21), 0, "cg"), ((15, 21), 0, "chebyshev"), ((15, 21), 0, "eyre_milton"),
         ((7, 9, 5), 1, "cg"), ((7, 9, 5), 1, "richardson"), ((9, 9, 9), 0, "cg")]


@pytest.mark.parametrize("N,rule,solver", CASES)
def test_history_matches_oracle(N, rule, solver):
    d = len(N)
    phase = I.paper_square(N)
    A = I.phase_to_full(phase, I.iso_tables(d, [1.0, 20.0]))
    Aop = orc.ga_assemble(N, A) if rule == 1 else A
    p = plan(N, A, rule)
    cap = 400
    h = p.set_history(cap)
    res, en = h["res"], h["energy"]
    E = np.zeros(d)
    E[0] = 1.0
    e, st, stats = p.solve(solver, E, 1e-8)
    m = stats[0]["iters"]
    assert st == 0 and 0 < m < cap
    ro = orc.solve(N, rule, Aop, E, solver, 1.0, 20.0, 1e-8, fixed_iters=m, energy=True)
    r_gpu = res[0, : m + 1].cpu().numpy()
    e_gpu = en[0, : m + 1].cpu().numpy()
    check_res(r_gpu, ro.res_hist)
    check_en(e_gpu, ro.energy_hist)
    assert torch.isnan(res[0, m + 1:]).all()  # nothing written past the last body
    # the final entries are what the solve reports
    bil, _ = p.effective(E, e)
    assert abs(e_gpu[m] - bil[0, 0]) <= 1e-12 * bil[0, 0]
    assert abs(r_gpu[m] - stats[0]["rel_res_recursive"]) <= 1e-12 * max(r_gpu[m], 1e-300)
    if rule == 1 and solver in ("cg", "richardson"):
        # Ga: the energy of the iterates never increases (Table 1; Sec. 4.3)
        assert np.all(np.diff(e_gpu) <= 1e-12 * e_gpu[0])


def test_history_ring_and_loads():
    """capacity below the body count keeps the latest entries at m mod capacity; load j writes row j."""
    N = (15, 15)
    A = I.phase_to_full(I.paper_square(N), I.iso_tables(2, [1.0, 20.0]))
    p = plan(N, A)
    h = p.set_history(500, nrhs=2)
    res_full, en_full = h["res"], h["energy"]
    E = np.eye(2)
    e, st, stats = p.solve("richardson", E, 1e-8)
    full_r = res_full.cpu().numpy()
    full_e = en_full.cpu().numpy()
    cap = 16
    h = p.set_history(cap, nrhs=2)
    res, en = h["res"], h["energy"]
    e2, st, stats2 = p.solve("richardson", E, 1e-8)
    r = res.cpu().numpy()
    g = en.cpu().numpy()
    for j in range(2):
        m = stats2[j]["iters"]
        assert m == stats[j]["iters"] and m > cap
        for k in range(m - cap + 1, m + 1):
            assert r[j, k % cap] == full_r[j, k]
            assert g[j, k % cap] == full_e[j, k]
    p.set_history(0)
    e3, _, _ = p.solve("richardson", E, 1e-8)
    assert torch.equal(e3, e2)


@pytest.mark.parametrize("solver", ["cg", "eyre_milton"])
def test_gani_bound_monitor(solver):
    """Energy history with a Ga plan: the guaranteed bound of every GaNi iterate, against the
    oracle's iterate prolonged and integrated exactly; it ends at fgh_gani_bound's value."""
    N = (15, 15)
    A = I.phase_to_full(I.paper_square(N), I.iso_tables(2, [1.0, 100.0]))
    gani = plan(N, A, 0)
    ga = plan(N, A, 1)
    en = gani.set_history(300, bound_plan=ga)["energy"]
    E = np.array([1.0, 0.0])
    e, st, stats = gani.solve(solver, E, 1e-6)
    m = stats[0]["iters"]
    assert st == 0 and m > 3
    got = en[0, : m + 1].cpu().numpy()
    AM = orc.ga_assemble(N, A)
    ref = [orc.energy(N, orc.GA, AM, E, None)]  # x_0 = 0 (EM: G_N E = 0): the Voigt bound
    for k in range(1, m + 1):
        ro = orc.solve(N, orc.GANI, A, E, solver, 1.0, 100.0, 1e-6, fixed_iters=k)
        ref.append(orc.energy(N, orc.GA, AM, E, orc.prolong(N, orc.project(N, orc.GANI, ro.e))))
    check_en(got, np.array(ref))
    gani.set_history(0)
    b = gani.gani_bound(ga, E, e)
    if solver == "cg":  # conforming iterate: the projection changes nothing beyond round-off
        assert abs(got[m] - b) <= 1e-11 * b
    # Ga energy of the Ga solution lies below every bound
    eg, _, _ = ga.solve("cg", E, 1e-10)
    bil, _ = ga.effective(E, eg)
    assert np.all(got >= bil[0, 0] * (1 - 1e-12))


def test_history_rejections():
    m = F()
    N = (9, 9)
    A = I.phase_to_full(I.paper_square(N), I.iso_tables(2, [1.0, 10.0]))
    p64 = plan(N, A, 0)
    p32 = plan(N, A, 0, precision=m.FGH_FP32_REFINED)
    ga = plan(N, A, 1)
    buf = torch.zeros(8, dtype=torch.float64, device="cuda")
    lib = m.lib()
    import ctypes
    h = lambda pl: ctypes.c_void_p(pl.handle)
    ptr = ctypes.c_void_p(buf.data_ptr())
    assert lib.fgh_plan_set_history(h(p32), ptr, ptr, None, None, None, 8, None) == m.FGH_E_UNSUPPORTED
    assert lib.fgh_plan_set_history(h(p64), ptr, ptr, None, None, None, 0, None) == m.FGH_E_INVALID
    assert lib.fgh_plan_set_history(h(ga), ptr, ptr, None, None, None, 8, h(ga)) == m.FGH_E_INVALID  # Ga monitored
    assert lib.fgh_plan_set_history(h(p64), ptr, None, None, None, None, 8, h(ga)) == m.FGH_E_INVALID  # bound: energy
    assert lib.fgh_plan_set_history(h(p64), None, None, ptr, None, None, 8, None) == m.FGH_E_INVALID  # no scratch
    assert lib.fgh_plan_set_history(h(p64), None, None, None, None, None, 0, None) == m.FGH_OK


@pytest.mark.parametrize("rule,solver", [(0, "eyre_milton"), (0, "cg"), (0, "richardson"), (1, "chebyshev")])
def test_nonconformity_history(rule, solver):
    """Sec. 4.4: ||G e_m - e_m|| and its mean-value part for every iterate, against the oracle's
    iterates (projection by the oracle's own G).  Eyre-Milton is non-conforming (large values,
    relative 1e-6); the conforming solvers stay at round-off (absolute 1e-12 |E|)."""
    N = (15, 21)
    A = I.phase_to_full(I.paper_square(N), I.iso_tables(2, [1.0, 20.0]))
    Aop = orc.ga_assemble(N, A) if rule == 1 else A
    p = plan(N, A, rule)
    h = p.set_history(200, conformity=True)
    E = np.array([1.0, 0.0])
    e, st, stats = p.solve(solver, E, 1e-6)
    m = stats[0]["iters"]
    assert st == 0 and 2 < m < 200
    nc = h["nonconf"][0, : m + 1].cpu().numpy()
    mn = h["mean"][0, : m + 1].cpu().numpy()
    g = orc.op_grid(N, rule)
    ref_nc, ref_mn = [], []
    for k in range(m + 1):
        if k == 0:
            ek = np.zeros((2,) + g)
        else:
            ek = orc.solve(N, rule, Aop, E, solver, 1.0, 20.0, 1e-6, fixed_iters=k).e
        gk = orc.project(N, rule, ek)
        ref_nc.append(np.sqrt(np.mean(np.sum((gk - ek) ** 2, axis=0))))
        ref_mn.append(np.linalg.norm(ek.reshape(2, -1).mean(axis=1)))
    ref_nc, ref_mn = np.array(ref_nc), np.array(ref_mn)
    if solver == "eyre_milton":
        assert np.all(np.abs(nc[1:] - ref_nc[1:]) <= 1e-6 * ref_nc[1:] + 1e-13), (nc, ref_nc)
        assert np.all(np.abs(mn[1:] - ref_mn[1:]) <= 1e-6 * ref_mn[1:] + 1e-13), (mn, ref_mn)
        assert np.all(mn <= nc * (1 + 1e-12))  # the mean part is one of two orthogonal parts
        assert nc[1] > 1e-4  # non-conforming from the first step on
    else:
        assert np.all(nc <= 1e-12) and np.all(ref_nc <= 1e-12), (nc, ref_nc)
        assert np.all(mn <= 1e-12) and np.all(ref_mn <= 1e-12), (mn, ref_mn)
