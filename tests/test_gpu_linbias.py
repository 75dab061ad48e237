"""Linear (non-local) bias, sections 2.2.1 and 2.4.1: gradient, Hessian-vector
product and MAP on the GPU against the oracle, through the C ABI, for the
lognormal and the Gaussian prior."""
import numpy as np
import pytest

from conftest import oracle_problem
from oracle import gaussian, linbias
from oracle import newton as o_newton
from oracle.grid import Problem, hermitian_weights, inv_lambda_half
from paper_0911_1407_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LN, GA = linbias.LOGNORMAL, linbias.GAUSSIAN


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _inst(n, cell, seed=0, inv_p0=0.5, nbar=1.3, sigma=1.0):
    box = tuple(cell * v for v in n)
    inst = synth.make_instance(n, box, sigma, nbar, 1.0, radius=0.45 * box[0], mask_frac=0.2, seed=seed, block=4)
    inst["inv_p0"] = inv_p0
    return inst


def _plan(inst, precision="fp64"):
    from paper_0911_1407_amd.binding import Plan
    p = Plan(inst["n"], inst["box"], precision=precision)
    p.set_instance(inst)
    return p


def _bk(inst, b0=0.9, smooth_cells=1.5):
    cell = inst["box"][0] / inst["n"][0]
    return synth.bias_multiplier_half(inst["n"], inst["box"], b0, smooth_cells * cell)


SHAPES = [((8, 8, 8), 8.0), ((16, 24, 32), 2.0), ((32, 32, 32), 4.0), ((48, 48, 48), 3.0)]


@pytest.mark.parametrize("kind", [LN, GA])
@pytest.mark.parametrize("n,cell", SHAPES)
def test_grad_and_hessvec_match_oracle(kind, n, cell):
    inst = _inst(n, cell)
    P = oracle_problem(inst)
    bk = _bk(inst)
    rng = np.random.default_rng(11)
    x = linbias.prior_mean(P, kind) + 0.3 * rng.standard_normal(n)
    v = rng.standard_normal(n)
    plan = _plan(inst, "mixed")
    bk_d = torch.from_numpy(bk).cuda()  # one device table: the HVP below reuses the linearisation
    g, obj = plan.linear_bias_grad(kind, bk_d, x)
    assert _rel(g.cpu().numpy(), linbias.gradient(P, bk, x, kind)) <= 1e-11
    assert obj == pytest.approx(linbias.objective(P, bk, x, kind), rel=1e-11)
    hv_ref = linbias.hessvec(P, bk, x, v, kind)
    hv = plan.linear_bias_hessvec(kind, bk_d, v).cpu().numpy()  # reuses the linearisation of the gradient
    assert _rel(hv, hv_ref) <= 1e-11
    hv2 = plan.linear_bias_hessvec(kind, bk_d, v, x=x).cpu().numpy()
    assert _rel(hv2, hv_ref) <= 1e-11


@pytest.mark.parametrize("kind", [LN, GA])
@pytest.mark.parametrize("n,cell", [((8, 8, 8), 8.0), ((16, 24, 32), 2.0), ((32, 32, 32), 4.0)])
def test_map_matches_oracle(kind, n, cell):
    # the lognormal posterior with a non-local bias need not be convex: with a
    # smoothing of 1.5 cells two local minima exist at 8^3 (seed 2); at one
    # cell the dense and the spectral oracle agree, so the MAP is unique here
    inst = _inst(n, cell, seed=2)
    P = oracle_problem(inst)
    bk = _bk(inst, 0.9, 1.0)
    ref, oinfo = linbias.newton_spectral(P, bk, kind, rtol=1e-11)
    assert oinfo["status"] == "ok", oinfo
    if np.prod(n) <= 512:
        dense, _ = linbias.map_dense(P, bk, kind, gtol_rel=1e-12)
        assert _rel(ref, dense) <= 1e-9
    plan = _plan(inst)
    x, info = plan.solve_linear_bias(kind, bk, rtol=1e-11, max_newton=200, max_cg=5000)
    assert info["status"] == 0 and info["rel_grad"] <= 1e-11, info
    assert _rel(x.cpu().numpy(), ref) <= 1e-7
    y = linbias.galaxy_field(P, bk, x.cpu().numpy(), kind)
    assert np.all(y[P.counts > 0] > 0)


def test_unit_multiplier_reproduces_unit_bias_solvers():
    # bk = 1 is the unit bias: the same MAP as the power-law solver at beta = 1
    # and as the unit-bias Gaussian-prior solver
    inst = _inst((32, 32, 32), 4.0, seed=5)
    one = np.ones(synth.hermitian_multiplicity(inst["n"]).shape)
    plan = _plan(inst)
    s_ln, info = plan.solve_linear_bias("lognormal", one, rtol=1e-11, max_cg=5000)
    assert info["status"] == 0, info
    s_ref, info_ref = plan.solve(rtol=1e-11, max_cg=5000, precision=0)
    assert info_ref["status"] == 0
    assert _rel(s_ln.cpu().numpy(), s_ref.cpu().numpy()) <= 1e-8
    d_ga, info = plan.solve_linear_bias("gaussian", one, rtol=1e-11, max_cg=5000)
    assert info["status"] == 0, info
    d_ref, info_ref = plan.solve_gaussian(rtol=1e-11, max_cg=5000, precision=0)
    assert info_ref["status"] == 0
    assert _rel(d_ga.cpu().numpy(), d_ref.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("kind,b0", [(LN, 1.0), (LN, 1.4), (GA, 0.7), (GA, 1.3)])
def test_white_prior_local_bias_closed_form(kind, b0):
    # S = sigma2 I and bk = b0 decouple the cells; per-cell roots by bisection
    n, box, sigma2, mu = (64, 64, 64), (128.0,) * 3, 0.6, -0.3
    inst = synth.make_instance(n, box, 1.0, 1.2, 1.0, radius=50.0, mask_frac=0.2, seed=3, block=8)
    inst.update(pk=np.full(inst["pk"].shape, sigma2 * np.prod(box) / np.prod(n)), amp=1.0, mu=mu,
                inv_p0=1.0 / sigma2)
    bk = np.full(inst["pk"].shape, b0)
    plan = _plan(inst)
    x, info = plan.solve_linear_bias(kind, bk, rtol=1e-12)
    assert info["status"] == 0, info
    m = mu if kind == LN else 0.0
    ref = linbias.white_prior_map(kind, sigma2, m, b0, inst["nbar"], inst["w"], inst["counts"])
    assert np.abs(x.cpu().numpy() - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("kind", [LN, GA])
def test_selection_workload_256_full_size(kind):
    # the 256^3 selection workload with a smoothing bias multiplier: every
    # output of the gradient and of one HVP against the oracle, then the MAP
    # to the benchmark tolerance, checked by the oracle's own gradient there
    inst = synth.config_instance("sel256")
    n = inst["n"]
    P = oracle_problem(inst)
    bk = _bk(inst, 1.0, 1.5)
    x0 = np.full(n, linbias.prior_mean(P, kind))
    rng = np.random.default_rng([0, 3])
    v = rng.standard_normal(n)
    print(f"linbias 256 kind={kind}: GPU operators", flush=True)
    plan = _plan(inst, "mixed")
    x_op = inst["s_true"] if kind == LN else np.expm1(inst["s_true"])
    bk_d = torch.from_numpy(bk).cuda()
    g, _ = plan.linear_bias_grad(kind, bk_d, x_op)
    hv = plan.linear_bias_hessvec(kind, bk_d, v)
    print("oracle operators", flush=True)
    # real-space operands: both sides carry the FFT roundoff of S^-1 applied
    # to a real field, eps times the 1/lambda spread (about 1e-10 at 256^3)
    assert _rel(g.cpu().numpy(), linbias.gradient(P, bk, x_op, kind)) <= 2e-9
    assert _rel(hv.cpu().numpy(), linbias.hessvec(P, bk, x_op, v, kind)) <= 2e-9
    print("GPU solve", flush=True)
    x, x_hat, info = plan.solve_linear_bias(kind, bk_d, want_hat=True, rtol=1e-6, max_cg=2000)
    assert info["status"] == 0 and info["rel_grad"] <= 1e-6, info
    print("oracle gradient at the GPU MAP", flush=True)
    xs = x.cpu().numpy()
    # the oracle's gradient in spectral form at the solver's spectral
    # iterate: S^-1 is an exact pointwise product there (section 2.3), so
    # there is no FFT-roundoff floor (a real field's high-k roundoff,
    # amplified by 1/lambda up to ~1e13, would put one near 4e-5 of g0)
    inv_lam = inv_lambda_half(P)
    m_hat = np.zeros(inv_lam.shape, dtype=np.complex128)
    m_hat[0, 0, 0] = P.ncells * linbias.prior_mean(P, kind)
    cw = hermitian_weights(n)

    def spectral_norm(xh):
        _, gh = linbias._spectral_grad(P, bk, xh, kind, inv_lam, m_hat)
        return np.sqrt(float(np.sum(cw * np.abs(gh) ** 2)) / P.ncells)

    g0 = spectral_norm(np.fft.rfftn(x0))
    gs = spectral_norm(x_hat.cpu().numpy())
    print(f"linbias 256 kind={kind}: oracle ||g||/||g0|| at the returned iterate {gs / g0:.3e}", flush=True)
    assert gs <= 1.01e-6 * g0
    # the k = 0 mode has 1/lambda = 0 (inv_p0 = 0), so its part of the MAP
    # equation is free of that floor: sum_i phi'(x)_i (B u)_i = 0 at the MAP,
    # to within sqrt(N) times the solve's tolerance on the gradient norm
    y = linbias.galaxy_field(P, bk, xs, kind)
    u = P.nbar * P.w - np.where(P.counts > 0, P.counts / y, 0.0)
    k0 = float(np.sum(linbias.dphi(kind, xs) * linbias.bias_apply(bk, u)))
    assert abs(k0) <= 1.01e-6 * np.sqrt(P.ncells) * g0
    assert np.all(y[P.counts > 0] > 0)


def test_error_paths():
    from paper_0911_1407_amd import binding
    inst = _inst((16, 16, 16), 4.0)
    bk = _bk(inst)
    bk_d = torch.from_numpy(bk).cuda()
    plan = _plan(inst)
    x = np.zeros(inst["n"])
    with pytest.raises(binding.PLError) as e:
        plan.linear_bias_hessvec("lognormal", bk, x)  # no linearisation yet
    assert "no_problem" in str(e.value)
    plan.linear_bias_grad("lognormal", bk_d, x)
    plan.linear_bias_hessvec("lognormal", bk_d, x)  # reuses it
    plan.grad(x)  # another call clears the cached linearisation
    with pytest.raises(binding.PLError) as e:
        plan.linear_bias_hessvec("lognormal", bk_d, x)
    assert "no_problem" in str(e.value)
    with pytest.raises(binding.PLError) as e:
        plan.linear_bias_grad(7, bk, x)
    assert "invalid_arg" in str(e.value)
    with pytest.raises(binding.PLError) as e:
        plan.solve_linear_bias("gaussian", bk, precision=1)
    assert "invalid_arg" in str(e.value)
    # the Gaussian prior from delta = -2 leaves y = 1 + B delta < 0 where there are counts
    with pytest.raises(binding.PLError) as e:
        plan.solve_linear_bias("gaussian", bk, x0=np.full(inst["n"], -2.0))
    assert "domain" in str(e.value)
    bad = bk.copy()
    bad[1, 1, 1] = np.nan
    with pytest.raises(binding.PLError) as e:
        plan.linear_bias_grad("gaussian", bad, x)
    assert "domain" in str(e.value)
    inst2 = dict(inst, beta=1.5)
    plan2 = _plan(inst2)
    with pytest.raises(binding.PLError) as e:
        plan2.linear_bias_grad("lognormal", bk, x)
    assert "invalid_arg" in str(e.value)
    # the plan still solves the power-law model afterwards
    s, info = plan.solve(rtol=1e-8, precision=0)
    assert info["status"] == 0


@pytest.mark.parametrize("kind", [LN, GA])
def test_no_data_returns_prior_mean(kind):
    # w = 0 and N = 0 everywhere: the likelihood vanishes, the gradient at the
    # prior mean is zero and the solve returns it after no iteration; from
    # another start with inv_p0 > 0 it reaches the prior mean
    inst = _inst((16, 16, 16), 4.0, inv_p0=0.5)
    inst["w"] = np.zeros(inst["n"])
    inst["counts"] = np.zeros(inst["n"])
    bk = _bk(inst)
    plan = _plan(inst)
    m = inst["mu"] if kind == LN else 0.0
    x, info = plan.solve_linear_bias(kind, bk, rtol=1e-10)
    assert info["status"] == 0 and info["newton_its"] == 0, info
    assert np.abs(x.cpu().numpy() - m).max() <= 1e-14
    x0 = m + 0.1 * np.random.default_rng(4).standard_normal(inst["n"])
    x, info = plan.solve_linear_bias(kind, bk, x0=x0, rtol=1e-12)
    assert info["status"] == 0, info
    assert np.abs(x.cpu().numpy() - m).max() <= 1e-10


@pytest.mark.parametrize("kind", [LN, GA])
def test_map_selection_workload_64_matches_oracle(kind):
    # the selection workload's recipe at 64^3 (radial selection, masked 8^3
    # blocks, nbar 0.5) with the benchmark's 1.5-cell smoothing multiplier;
    # oracle Newton paths with different preconditioners reach the same
    # minimiser on this recipe (asserted on the CPU by
    # test_oracle_spectral.test_linear_bias_minimiser_does_not_depend_on_preconditioner),
    # so the comparison is of the MAP itself
    inst = synth.config_instance("sel256", n=64)
    P = oracle_problem(inst)
    bk = _bk(inst, 1.0, 1.5)
    print(f"linbias 64 kind={kind}: oracle", flush=True)
    ref, oinfo = linbias.newton_spectral(P, bk, kind, rtol=1e-10)
    assert oinfo["status"] == "ok", oinfo
    plan = _plan(inst)
    x, info = plan.solve_linear_bias(kind, bk, rtol=1e-10, max_cg=5000)
    assert info["status"] == 0 and info["rel_grad"] <= 1e-10, info
    assert _rel(x.cpu().numpy(), ref) <= 1e-7
