"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Outputs are compared as a whole (relative L2) and element by element
(``assert_elementwise``: every entry within the tolerance of the oracle's, in
units of max(|ref|, floor * max|ref|)).  Tolerances: FP64 operators 1e-11 relative (FFT roundoff times the spread of
1/lambda); FP64 MAP rel-L2 1e-6 against the oracle MAP solved to 1e-11 (both
sides are solved tighter, so the observed gap is far smaller); mixed
FP32/FP64 MAP rel-L2 1e-4; FP32 operators 2e-5 relative.
"""
import numpy as np
import pytest

from conftest import assert_elementwise, oracle_problem
from oracle import adjoint as o_adj
from oracle import model as o_model
from oracle import newton as o_newton
from oracle.grid import Problem
from paper_0911_1407_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _plan(inst, precision="fp64"):
    from paper_0911_1407_amd.binding import Plan
    p = Plan(inst["n"], inst["box"], precision=precision)
    p.set_instance(inst)
    return p


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


# grids: several tiles, ragged column tiles (odd nz/2+1), mixed lengths
OPERATOR_GRIDS = [
    (8, 8, 8), (12, 12, 12), (16, 16, 16), (24, 24, 24), (32, 32, 32), (48, 48, 48), (64, 64, 64),
    (96, 96, 96), (128, 128, 128), (16, 24, 32), (48, 32, 12), (8, 64, 96), (192, 16, 24),
]


def _inst(n, beta=1.3, seed=0, mask=0.2, coarse=True):
    # coarse cells keep 1/lambda within a few decades so operator parity is
    # not limited by the prior's conditioning
    cell = 8.0 if coarse else 2.0
    box = tuple(cell * v for v in n)
    blk = 4 if min(n) % 4 == 0 and min(n) >= 8 else 2
    return synth.make_instance(n, box, 1.2, 1.1, beta, radius=0.4 * box[0], mask_frac=mask, seed=seed,
                               block=blk)


@pytest.mark.parametrize("n", OPERATOR_GRIDS)
def test_grad_and_hessvec_match_oracle(n):
    inst = _inst(n)
    P = oracle_problem(inst)
    rng = np.random.default_rng(5)
    s = inst["s_true"] + 0.05 * rng.standard_normal(n)
    v = rng.standard_normal(n)
    plan = _plan(inst)
    g, obj = plan.grad(s)
    g_ref = o_model.gradient(P, s)
    assert _rel(_np(g), g_ref) <= 1e-11
    assert_elementwise(_np(g), g_ref, 1e-10, what=f"gradient {n}")
    assert abs(obj - o_model.objective(P, s)) <= 1e-11 * abs(o_model.objective(P, s))
    hv = plan.hessvec(v)  # cached diagonal from pl_grad
    hv_ref = o_model.hessvec(P, s, v)
    assert _rel(_np(hv), hv_ref) <= 1e-11
    assert_elementwise(_np(hv), hv_ref, 1e-10, what=f"HVP {n}")
    hv2 = plan.hessvec(v, s=s)
    assert _rel(_np(hv2), hv_ref) <= 1e-11


def test_prior_table_radial_and_per_mode():
    # an isotropic spectrum on a cubic box runs on the radial shell table; a
    # spectrum off by 1e-12 at one mode (or a non-cubic box) on the per-mode
    # table; both match the oracle, which always applies pk mode by mode
    from paper_0911_1407_amd import binding
    rng = np.random.default_rng(8)
    for n, box_scale, perturb, radial in (((32, 32, 32), (8, 8, 8), False, True),
                                          ((32, 32, 32), (8, 8, 8), True, False),
                                          ((32, 32, 32), (8, 8, 6), False, False)):
        box = tuple(b * v for b, v in zip(box_scale, n))
        inst = synth.make_instance(n, box, 1.2, 1.1, 1.3, radius=0.4 * box[0], mask_frac=0.2, seed=3, block=4)
        if perturb:
            inst["pk"] = inst["pk"].copy()
            inst["pk"][3, 5, 7] *= 1.0 + 1e-12
        plan = _plan(inst)
        assert binding.pl_plan_prior_is_radial(plan.h) == radial
        P = oracle_problem(inst)
        s = inst["s_true"] + 0.05 * rng.standard_normal(n)
        v = rng.standard_normal(n)
        g, _ = plan.grad(s)
        assert _rel(_np(g), o_model.gradient(P, s)) <= 1e-11
        assert _rel(_np(plan.hessvec(v)), o_model.hessvec(P, s, v)) <= 1e-11


@pytest.mark.parametrize("n", [(32, 32, 32), (48, 48, 48), (16, 24, 32), (96, 96, 96)])
def test_hessvec_f32_matches_oracle(n):
    inst = _inst(n)
    P = oracle_problem(inst)
    rng = np.random.default_rng(6)
    s = inst["s_true"]
    v = rng.standard_normal(n).astype(np.float32)
    plan = _plan(inst, "mixed")
    hv = plan.hessvec_f32(v, s=s)
    hv_ref = o_model.hessvec(P, s, v.astype(np.float64))
    assert _rel(_np(hv).astype(np.float64), hv_ref) <= 2e-5
    assert_elementwise(_np(hv).astype(np.float64), hv_ref, 2e-4, what=f"FP32 HVP {n}")


@pytest.mark.parametrize("n", [(32, 32, 32), (64, 64, 64), (16, 24, 32)])
def test_spectral_hessvec_matches_oracle(n):
    inst = _inst(n)
    P = oracle_problem(inst)
    rng = np.random.default_rng(7)
    s = inst["s_true"]
    v = rng.standard_normal(n)
    v_hat = np.fft.rfftn(v)
    plan = _plan(inst, "mixed")
    plan.grad(s)
    ref = o_newton.SpectralOps(P).hessvec(o_model.hess_diag(P, s), v_hat)
    out = plan.hessvec_hat(torch.from_numpy(v_hat).cuda())
    assert np.linalg.norm(_np(out) - ref) <= 1e-11 * np.linalg.norm(ref)
    assert_elementwise(_np(out), ref, 1e-10, what=f"spectral HVP {n}")
    out32 = plan.hessvec_hat(torch.from_numpy(v_hat.astype(np.complex64)).cuda())
    assert np.linalg.norm(_np(out32) - ref) <= 2e-5 * np.linalg.norm(ref)
    assert_elementwise(_np(out32), ref, 2e-4, what=f"spectral FP32 HVP {n}")


@pytest.mark.parametrize("n,beta", [((8, 8, 8), 1.3), ((16, 16, 16), 1.0), ((24, 16, 32), 1.5), ((48, 48, 48), 1.2)])
def test_map_matches_oracle_fp64(n, beta):
    inst = _inst(n, beta=beta, coarse=False)
    P = oracle_problem(inst)
    s_ref, info_ref = o_newton.newton_krylov(P, rtol=1e-11)
    plan = _plan(inst)
    s, info = plan.solve(rtol=1e-11)
    assert info["status"] == 0, info
    assert _rel(_np(s), s_ref) <= 1e-6
    assert_elementwise(_np(s), s_ref, 1e-6, what=f"MAP {n}")
    assert info["rel_grad"] <= 1e-11


def test_map_plain32_workload():
    # 32^3, box 100 Mpc/h, sigma_G = 1, unit bias, w = 1, nbar = 1, rtol 1e-8
    inst = synth.config_instance("plain32")
    P = oracle_problem(inst)
    s_ref, _ = o_newton.newton_krylov(P, rtol=1e-11)
    for prec in ("fp64", "mixed"):
        plan = _plan(inst, prec)
        s, info = plan.solve(rtol=1e-8)
        assert info["status"] == 0, (prec, info)
        assert info["rel_grad"] <= 1e-8
        tol = 1e-6 if prec == "fp64" else 1e-4
        assert _rel(_np(s), s_ref) <= tol, prec
        assert_elementwise(_np(s), s_ref, tol, what=f"plain32 MAP {prec}")
        print(f"plain32 {prec} rtol 1e-8: rel-L2 vs oracle {_rel(_np(s), s_ref):.3e}, fp64 steps "
              f"{info['fp64_steps']}", flush=True)


def test_white_prior_closed_form_on_gpu():
    from oracle import closed_form
    n, box, sigma2 = (64, 64, 64), (128.0,) * 3, 0.7
    inst = synth.make_instance(n, box, 1.0, 0.8, 1.4, radius=50.0, mask_frac=0.2, seed=3, block=8)
    ncell = np.prod(n)
    pk = np.full(inst["pk"].shape, sigma2 * np.prod(box) / ncell)
    plan = _plan(inst)
    plan.set_problem(inst["w"], inst["counts"], pk, 1.0, -0.3, 0.8, 1.4, 1.0 / sigma2)
    s, info = plan.solve(rtol=1e-12)
    ref = closed_form.white_prior_map(mu=-0.3, sigma2=sigma2, beta=1.4, nbar=0.8, w=inst["w"],
                                      counts=inst["counts"])
    assert _rel(_np(s), ref) <= 1e-10


def test_zero_completeness_and_uniform_data():
    from oracle import closed_form
    n, box = (32, 32, 32), (64.0,) * 3
    inst = synth.make_instance(n, box, 1.0, 1.0, 1.0, seed=0)
    plan = _plan(inst)
    plan.set_problem(np.zeros(n), np.zeros(n), inst["pk"], inst["amp"], -0.5, 2.0, 1.0, 0.0)
    rng = np.random.default_rng(1)
    s0 = -0.5 + 0.3 * rng.standard_normal(n)
    s, info = plan.solve(s0=s0, rtol=1e-12)
    assert np.abs(_np(s) - closed_form.zero_completeness_map(s0, -0.5, 0.0)).max() <= 1e-9
    s, info = plan.solve(rtol=1e-12)
    assert info["newton_its"] == 0 and np.all(_np(s) == -0.5)
    plan.set_problem(np.full(n, 0.3), np.full(n, 3.0), inst["pk"], inst["amp"], -0.5, 2.0, 1.6, 0.0)
    s, info = plan.solve(rtol=1e-13)
    assert np.abs(_np(s) - closed_form.uniform_data_map(3.0, 2.0, 0.3, 1.6)).max() <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adjoint_matches_oracle(prec):
    # 2 Mpc/h cells: cond(H) ~ 1e16, so the reference is the oracle's
    # spectral PCG adjoint (pinned to central differences; a dense real-space
    # solve loses ~1e-4 to the conditioning here)
    n = (16, 16, 16)
    inst = _inst(n, beta=1.5, coarse=False)
    P = oracle_problem(inst)
    s_ref, _ = o_newton.newton_krylov(P, rtol=1e-12)
    _, dL_ref = o_adj.squared_error_loss(s_ref, inst["s_true"])
    lam_ref, _ = o_adj.adjoint_pcg(P, s_ref, dL_ref, rtol=1e-13, max_cg=5000)
    gr_ref = o_adj.param_grads(P, s_ref, lam_ref)
    plan = _plan(inst, prec)
    s, info = plan.solve(rtol=1e-12, precision=0)
    _, dL = o_adj.squared_error_loss(_np(s), inst["s_true"])
    grads, ainfo = plan.adjoint(s, dL, rtol=1e-12 if prec == "fp64" else 1e-6, max_cg=5000)
    assert ainfo["status"] == 0, ainfo
    tol = 1e-6 if prec == "fp64" else 1e-4
    assert _rel(_np(grads["lam"]), lam_ref) <= tol
    assert_elementwise(_np(grads["lam"]), lam_ref, tol, what=f"adjoint lambda {prec}")
    for k in ("A", "beta", "nbar"):
        assert abs(grads[k] - gr_ref[k]) <= tol * abs(gr_ref[k]), k
    assert _rel(_np(grads["N"]), gr_ref["N"]) <= tol
    assert _rel(_np(grads["w"]), gr_ref["w"]) <= tol


def test_adjoint_dense_reference_well_conditioned():
    # coarse cells keep cond(H) small enough for the dense real-space solve
    n = (8, 8, 8)
    inst = _inst(n, beta=1.3, coarse=True)
    P = oracle_problem(inst)
    s_ref, _ = o_newton.newton_dense(P)
    _, dL_ref = o_adj.squared_error_loss(s_ref, inst["s_true"])
    gr_ref = o_adj.param_grads(P, s_ref, o_adj.adjoint_dense(P, s_ref, dL_ref))
    plan = _plan(inst)
    s, _ = plan.solve(rtol=1e-13)
    _, dL = o_adj.squared_error_loss(_np(s), inst["s_true"])
    grads, ainfo = plan.adjoint(s, dL, rtol=1e-13, max_cg=5000)
    for k in ("A", "beta", "nbar"):
        assert abs(grads[k] - gr_ref[k]) <= 1e-8 * abs(gr_ref[k]), k


def test_adjoint_matches_central_fd_bias_workload():
    # the bias workload (beta = 1.5, nbar = 2, radial selection, 20% masked
    # 8^3 blocks) at 32^3 with the same cell size; loss sum (s* - s_true)^2;
    # central differences with relative step 1e-5 through GPU forward solves
    inst = synth.config_instance("bias256", n=32)
    plan = _plan(inst)
    st = inst["s_true"]

    def loss(**over):
        prm = dict(w=inst["w"], counts=inst["counts"], pk=inst["pk"], amp=inst["amp"], mu=inst["mu"],
                   nbar=inst["nbar"], beta=inst["beta"], inv_p0=0.0)
        prm.update(over)
        plan.set_problem(**prm)
        s, info = plan.solve(rtol=1e-13, max_newton=200, max_cg=2000)
        assert info["status"] == 0, info
        return float(np.sum((_np(s) - st) ** 2)), s

    L0, s_star = loss()
    grads, ainfo = plan.adjoint(s_star, 2.0 * (_np(s_star) - st), rtol=1e-13, max_cg=5000)
    for key, name in (("amp", "A"), ("beta", "beta"), ("nbar", "nbar")):
        v = inst[key]
        h = 1e-5 * v
        fd = (loss(**{key: v + h})[0] - loss(**{key: v - h})[0]) / (2 * h)
        assert abs(grads[name] - fd) <= 1e-5 * abs(fd), (name, grads[name], fd)
    plan.set_instance(inst)
    grads, _ = plan.adjoint(s_star, 2.0 * (_np(s_star) - st), rtol=1e-13, max_cg=5000)
    # direction of +-1 on cells with counts > 0 (counts must stay >= 0)
    u = np.random.default_rng(3).choice([-1.0, 1.0], size=inst["n"]) * (inst["counts"] > 0)
    fd = (loss(counts=inst["counts"] + 1e-5 * u)[0] - loss(counts=inst["counts"] - 1e-5 * u)[0]) / 2e-5
    assert abs(float(np.sum(_np(grads["N"]) * u)) - fd) <= 1e-5 * abs(fd)


def test_error_paths():
    from paper_0911_1407_amd import binding
    n = (16, 16, 16)
    inst = _inst(n)
    plan = _plan(inst)
    bad = inst["counts"].copy()
    bad[0, 0, 0] = -1
    with pytest.raises(binding.PLError) as e:
        plan.set_problem(inst["w"], bad, inst["pk"], inst["amp"], inst["mu"], inst["nbar"])
    assert e.value.code == binding.PL_ERR_DOMAIN
    w0 = inst["w"].copy()
    idx = np.argwhere(inst["counts"] > 0)[0]
    w0[tuple(idx)] = 0.0
    with pytest.raises(binding.PLError) as e:
        plan.set_problem(w0, inst["counts"], inst["pk"], inst["amp"], inst["mu"], inst["nbar"])
    assert e.value.code == binding.PL_ERR_DOMAIN
    nan_counts = inst["counts"].copy()
    nan_counts[1, 2, 3] = np.nan
    with pytest.raises(binding.PLError) as e:
        plan.set_problem(inst["w"], nan_counts, inst["pk"], inst["amp"], inst["mu"], inst["nbar"])
    assert e.value.code == binding.PL_ERR_DOMAIN
    pk0 = inst["pk"].copy()
    pk0[1, 0, 0] = 0.0
    with pytest.raises(binding.PLError) as e:
        plan.set_problem(inst["w"], inst["counts"], pk0, inst["amp"], inst["mu"], inst["nbar"])
    assert e.value.code == binding.PL_ERR_DOMAIN
    plan.set_instance(inst)
    s, info = plan.solve(rtol=1e-10, max_newton=1)
    assert info["status"] == binding.PL_ERR_NOT_CONVERGED and info["newton_its"] == 1
