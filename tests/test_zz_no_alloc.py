"""The allocation-free apply (fgh_apply_noalloc) against the plan-based fgh_apply, through the
C-ABI: two calls in a row on one GPU, the second on a smaller grid (the scratch array keeps the
first call's contents), to the FP64 operator tolerance 1e-12; plus the size limit."""
import numpy as np
import pytest

from paper_1508_02045_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_02045_amd import fgh
    fgh.lib()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(N, kind, seed):
    from paper_1508_02045_amd import fgh
    d = len(N)
    rng = np.random.default_rng(seed)
    if kind == "phase":
        ph, _, _ = I.boolean_spheres(N, 3.0, 0.3, rng)
        tab = np.stack([I.sym_pack(t[None])[:, 0] for t in I.iso_tables(d, [1.0, 50.0])])
        args = dict(a_kind=fgh.FGH_A_PHASE, A=None, phase=torch.from_numpy(ph).cuda(), phase_table=tab)
        plan = fgh.Plan(N, phase=args["phase"], phase_table=tab)
    else:
        A = torch.from_numpy(I.sym_pack(I.anisotropic_field(N, rng, 1.0, 30.0))).cuda()
        args = dict(a_kind=fgh.FGH_A_SYM, A=A, phase=None, phase_table=None)
        plan = fgh.Plan(N, A=A, a_kind=fgh.FGH_A_SYM)
    x = torch.from_numpy(rng.standard_normal((d,) + tuple(N))).cuda()
    return plan, args, x


@pytest.mark.parametrize("cases", [[((45, 63, 81), "phase"), ((27, 25, 21), "sym")],
                                   [((81, 81), "sym"), ((21, 15), "phase")]])
def test_noalloc_apply_matches_plan_apply_twice(cases):
    from paper_1508_02045_amd import fgh
    for k, (N, kind) in enumerate(cases):
        print(f"no-alloc apply call {k + 1}: N={N} kind={kind}", flush=True)
        plan, args, x = _case(N, kind, 11 + k)
        y_ref = plan.apply(x)
        y = torch.full_like(x, float("nan"))
        fgh.fgh_apply_noalloc(len(N), N, args["a_kind"], args["A"], args["phase"], args["phase_table"], x, y,
                              torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        yn, yr = y.cpu().numpy(), y_ref.cpu().numpy()
        assert np.isfinite(yn).all()
        assert rel(yn, yr) <= 1e-12, (N, kind, rel(yn, yr))
        plan.close()


def test_noalloc_apply_rejects_grids_beyond_the_scratch_array():
    from paper_1508_02045_amd import fgh
    N = (135, 135, 135)
    x = torch.zeros((3, 1), dtype=torch.float64, device="cuda")  # never read: the size check comes first
    ph = torch.zeros(1, dtype=torch.uint8, device="cuda")
    tab = np.array([[1.0, 0, 0, 1, 0, 1]])
    with pytest.raises(fgh.FghError) as ei:
        fgh.fgh_apply_noalloc(3, N, fgh.FGH_A_PHASE, None, ph, tab, x, x, torch.cuda.current_stream().cuda_stream)
    assert ei.value.status == fgh.FGH_E_WORKSPACE
