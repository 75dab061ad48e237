"""The allocation-free entry point (pl_compare_fields_noalloc, device scratch
held by the library) against the plan-based pl_compare_fields, through the C
ABI: two calls in a row, the second on a smaller grid, so the second call
must not see the first one's partial sums."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _fields(n, seed):
    rng = np.random.default_rng(seed)
    ref = rng.standard_normal(n)
    rec = 0.8 * ref + 0.3 * rng.standard_normal(n)
    return torch.from_numpy(rec).cuda(), torch.from_numpy(ref).cuda()


def test_noalloc_compare_matches_plan_entry_point():
    from paper_0911_1407_amd import binding
    from paper_0911_1407_amd.binding import Plan
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n, seed in (((64, 48, 32), 1), ((16, 24, 8), 2)):
        rec, ref = _fields(n, seed)
        plan = Plan(n, tuple(2.0 * v for v in n), precision="fp64")
        r_plan, d_plan = plan.compare(rec, ref)
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        binding.pl_compare_fields_noalloc(n, rec, ref, out, stream)
        torch.cuda.synchronize()
        r, d = out.cpu().tolist()
        print(f"n={n}: noalloc r={r!r} D={d!r}; plan r={r_plan!r} D={d_plan!r}", flush=True)
        # same kernels, same fixed summation order: equal to rounding of the
        # final division and square roots
        assert abs(r - r_plan) <= 4e-16 * abs(r_plan)
        assert abs(d - d_plan) <= 4e-16 * abs(d_plan)
        # against numpy in FP64
        a, b = rec.cpu().numpy().ravel(), ref.cpu().numpy().ravel()
        assert r == pytest.approx(float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b))), rel=1e-13)
        assert d == pytest.approx(float(np.sqrt(np.mean((a - b) ** 2))), rel=1e-13)
        plan.close()


def test_noalloc_compare_zero_field_and_bad_sizes():
    from paper_0911_1407_amd import binding
    n = (8, 8, 8)
    rec = torch.zeros(n, dtype=torch.float64, device="cuda")
    ref = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    binding.pl_compare_fields_noalloc(n, rec, ref, out)
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [0.0, 1.0]
    for bad, code in (((1024, 512, 512), binding.PL_ERR_UNSUPPORTED_SIZE), ((0, 8, 8), binding.PL_ERR_INVALID_ARG)):
        with pytest.raises(binding.PLError) as e:
            binding.pl_compare_fields_noalloc(bad, rec, ref, out)
        assert e.value.code == code
