"""Thin Python binding of libpl.so (argument marshalling only).

Every computation runs in the HIP library; this module only converts torch
device tensors to pointers and back.  Functions carry the names of the C ABI
declared in include/pl.h.  If libpl.so has not been built, ``load()`` raises:
there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpl.so")

PL_OK = 0
PL_ERR_INVALID_ARG = 1
PL_ERR_DOMAIN = 2
PL_ERR_UNSUPPORTED_SIZE = 3
PL_ERR_NOT_CONVERGED = 4
PL_ERR_LINESEARCH = 5
PL_ERR_HIP = 6
PL_ERR_NO_PROBLEM = 7
PL_FP64 = 0
PL_MIXED = 1

STATUS_NAMES = {0: "ok", 1: "invalid_arg", 2: "domain", 3: "unsupported_size", 4: "not_converged",
                5: "linesearch", 6: "hip", 7: "no_problem"}

SUPPORTED_LENGTHS = (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 512)

EXPORTED = ("pl_default_opts", "pl_plan_create", "pl_plan_set_workspace", "pl_plan_set_stream",
            "pl_plan_destroy", "pl_set_problem", "pl_grad", "pl_hessvec", "pl_hessvec_f32",
            "pl_hessvec_hat", "pl_hessvec_hat_f32", "pl_newton_krylov_solve", "pl_solve_adjoint",
            "pl_last_error", "pl_batch_create", "pl_batch_set_workspace", "pl_batch_set_problem",
            "pl_batch_solve", "pl_batch_destroy", "pl_batch_last_error", "pl_plan_autotune",
            "pl_plan_get_variants", "pl_plan_set_variants", "pl_plan_prior_is_radial", "pl_lsq_solve", "pl_nlcg_solve", "pl_lognormal_prior",
            "pl_gaussian_map_solve",
            "pl_inverse_weight", "pl_compare_fields", "pl_linear_bias_grad", "pl_linear_bias_hessvec",
            "pl_linear_bias_solve", "pl_newton_krylov_solve_hat", "pl_linear_bias_solve_hat",
            "pl_compare_fields_noalloc", "pl_batch_autotune")

# priors of the linear-bias calls (PL_MODEL_* in pl.h)
MODEL_LOGNORMAL = 0
MODEL_GAUSSIAN = 1
MODELS = {"lognormal": MODEL_LOGNORMAL, "gaussian": MODEL_GAUSSIAN}

BATCH_LENGTHS = (32, 48, 64, 96, 128)


class PLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class pl_problem(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("counts", ctypes.c_void_p), ("pk", ctypes.c_void_p),
                ("amp", ctypes.c_double), ("mu", ctypes.c_double), ("nbar", ctypes.c_double),
                ("beta", ctypes.c_double), ("inv_p0", ctypes.c_double)]


class pl_solve_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_newton", ctypes.c_int), ("max_cg", ctypes.c_int),
                ("eta_max", ctypes.c_double), ("ls_c1", ctypes.c_double), ("precision", ctypes.c_int),
                ("check_every", ctypes.c_int)]


class pl_solve_info(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int), ("cg_its", ctypes.c_int), ("hvps", ctypes.c_int),
                ("status", ctypes.c_int), ("rel_grad", ctypes.c_double), ("grad0", ctypes.c_double),
                ("obj", ctypes.c_double), ("fp64_steps", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_} | {"status_name": STATUS_NAMES.get(self.status)}


_lib = None


def load(path=LIB_PATH):
    """Load libpl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpl.so not found at {path}: build it with "
                           f"`python -m paper_0911_1407_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.pl_default_opts.argtypes = [ctypes.POINTER(pl_solve_opts)]
    lib.pl_default_opts.restype = None
    lib.pl_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(dbl), i32, vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.pl_plan_set_workspace.argtypes = [vp, vp]
    lib.pl_plan_set_stream.argtypes = [vp, vp]
    lib.pl_plan_destroy.argtypes = [vp]
    lib.pl_set_problem.argtypes = [vp, ctypes.POINTER(pl_problem)]
    lib.pl_grad.argtypes = [vp, vp, vp, ctypes.POINTER(dbl)]
    lib.pl_hessvec.argtypes = [vp, vp, vp, vp]
    lib.pl_hessvec_f32.argtypes = [vp, vp, vp, vp]
    lib.pl_hessvec_hat.argtypes = [vp, vp, vp]
    lib.pl_hessvec_hat_f32.argtypes = [vp, vp, vp]
    lib.pl_newton_krylov_solve.argtypes = [vp, vp, ctypes.POINTER(pl_solve_opts), ctypes.POINTER(pl_solve_info)]
    lib.pl_newton_krylov_solve_hat.argtypes = [vp, vp, vp, ctypes.POINTER(pl_solve_opts),
                                               ctypes.POINTER(pl_solve_info)]
    lib.pl_solve_adjoint.argtypes = [vp, vp, vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                     ctypes.POINTER(dbl), vp, vp, ctypes.POINTER(pl_solve_opts),
                                     ctypes.POINTER(pl_solve_info)]
    lib.pl_last_error.argtypes = [vp]
    lib.pl_last_error.restype = ctypes.c_char_p
    lib.pl_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(dbl), i32, vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.pl_batch_set_workspace.argtypes = [vp, vp]
    lib.pl_batch_set_problem.argtypes = [vp, i32, ctypes.POINTER(pl_problem)]
    lib.pl_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(pl_solve_opts),
                                   ctypes.POINTER(pl_solve_info)]
    lib.pl_batch_autotune.argtypes = [vp, ctypes.c_char_p]
    lib.pl_batch_destroy.argtypes = [vp]
    lib.pl_plan_autotune.argtypes = [vp, ctypes.c_char_p]
    lib.pl_plan_get_variants.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.pl_plan_prior_is_radial.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.pl_lsq_solve.argtypes = [vp, vp, ctypes.POINTER(pl_solve_opts), ctypes.POINTER(pl_solve_info)]
    lib.pl_nlcg_solve.argtypes = [vp, vp, ctypes.POINTER(pl_solve_opts), ctypes.POINTER(pl_solve_info)]
    lib.pl_gaussian_map_solve.argtypes = [vp, vp, ctypes.POINTER(pl_solve_opts), ctypes.POINTER(pl_solve_info)]
    lib.pl_lognormal_prior.argtypes = [vp, vp, ctypes.c_double, vp, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.pl_inverse_weight.argtypes = [vp, vp]
    lib.pl_compare_fields.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.pl_compare_fields_noalloc.argtypes = [ctypes.POINTER(ctypes.c_int32), vp, vp, vp, vp]
    lib.pl_plan_set_variants.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.pl_linear_bias_grad.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(dbl)]
    lib.pl_linear_bias_hessvec.argtypes = [vp, i32, vp, vp, vp, vp]
    lib.pl_linear_bias_solve.argtypes = [vp, i32, vp, vp, ctypes.POINTER(pl_solve_opts),
                                         ctypes.POINTER(pl_solve_info)]
    lib.pl_linear_bias_solve_hat.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(pl_solve_opts),
                                             ctypes.POINTER(pl_solve_info)]
    lib.pl_batch_last_error.argtypes = [vp]
    lib.pl_batch_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("pl_default_opts", "pl_last_error", "pl_batch_last_error"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(plan_handle, rc, allow=()):
    if rc != PL_OK and rc not in allow:
        msg = load().pl_last_error(plan_handle).decode() if plan_handle else ""
        raise PLError(rc, msg)
    return rc


# ---------------------------------------------------------------------------
# C-named functions
# ---------------------------------------------------------------------------

def pl_default_opts():
    o = pl_solve_opts()
    load().pl_default_opts(ctypes.byref(o))
    return o


def pl_plan_create(n, box, precision=PL_FP64, stream=None):
    """Returns (handle, workspace_bytes)."""
    lib = load()
    h = ctypes.c_void_p()
    nn = (ctypes.c_int32 * 3)(*[int(v) for v in n])
    bb = (ctypes.c_double * 3)(*[float(v) for v in box])
    ws = ctypes.c_size_t()
    rc = lib.pl_plan_create(ctypes.byref(h), nn, bb, int(precision), stream, ctypes.byref(ws))
    if rc != PL_OK:
        raise PLError(rc, f"pl_plan_create(n={tuple(n)}, box={tuple(box)})")
    return h, ws.value


def pl_plan_set_workspace(h, ws_tensor):
    return _check(h, load().pl_plan_set_workspace(h, _ptr(ws_tensor)))


def pl_plan_set_stream(h, stream):
    return _check(h, load().pl_plan_set_stream(h, stream))


def pl_plan_destroy(h):
    return load().pl_plan_destroy(h)


def pl_set_problem(h, w, counts, pk, amp, mu, nbar, beta=1.0, inv_p0=0.0):
    pr = pl_problem(_ptr(w).value, _ptr(counts).value, _ptr(pk).value, float(amp), float(mu), float(nbar),
                    float(beta), float(inv_p0))
    return _check(h, load().pl_set_problem(h, ctypes.byref(pr)))


def pl_grad(h, s, grad_out, want_obj=True):
    obj = ctypes.c_double()
    _check(h, load().pl_grad(h, _ptr(s), _ptr(grad_out), ctypes.byref(obj) if want_obj else None))
    return obj.value if want_obj else None


def pl_hessvec(h, s, v, hv_out):
    return _check(h, load().pl_hessvec(h, _ptr(s), _ptr(v), _ptr(hv_out)))


def pl_hessvec_f32(h, s, v, hv_out):
    return _check(h, load().pl_hessvec_f32(h, _ptr(s), _ptr(v), _ptr(hv_out)))


def pl_hessvec_hat(h, v_hat, hv_hat):
    return _check(h, load().pl_hessvec_hat(h, _ptr(v_hat), _ptr(hv_hat)))


def pl_hessvec_hat_f32(h, v_hat, hv_hat):
    return _check(h, load().pl_hessvec_hat_f32(h, _ptr(v_hat), _ptr(hv_hat)))


def pl_newton_krylov_solve(h, s_inout, opts=None):
    info = pl_solve_info()
    rc = load().pl_newton_krylov_solve(h, _ptr(s_inout), ctypes.byref(opts) if opts else None,
                                       ctypes.byref(info))
    _check(h, rc, allow=(PL_ERR_NOT_CONVERGED, PL_ERR_LINESEARCH))
    return info


def pl_newton_krylov_solve_hat(h, s_inout, s_hat_out, opts=None):
    info = pl_solve_info()
    rc = load().pl_newton_krylov_solve_hat(h, _ptr(s_inout), _ptr(s_hat_out), ctypes.byref(opts) if opts else None,
                                           ctypes.byref(info))
    _check(h, rc, allow=(PL_ERR_NOT_CONVERGED, PL_ERR_LINESEARCH))
    return info


def pl_solve_adjoint(h, s_star, dL_ds, lambda_out=None, dL_dN=None, dL_dw=None, opts=None):
    dA, db, dn = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    info = pl_solve_info()
    rc = load().pl_solve_adjoint(h, _ptr(s_star), _ptr(dL_ds), _ptr(lambda_out), ctypes.byref(dA),
                                 ctypes.byref(db), ctypes.byref(dn), _ptr(dL_dN), _ptr(dL_dw),
                                 ctypes.byref(opts) if opts else None, ctypes.byref(info))
    _check(h, rc, allow=(PL_ERR_NOT_CONVERGED,))
    return {"A": dA.value, "beta": db.value, "nbar": dn.value}, info


def pl_last_error(h):
    return load().pl_last_error(h).decode()


def pl_plan_autotune(h, cache_path=None):
    return _check(h, load().pl_plan_autotune(h, cache_path.encode() if cache_path else None))


def pl_lognormal_prior(h, pk, amp, pk_log_out):
    mu = ctypes.c_double(0.0)
    s0 = ctypes.c_double(0.0)
    nc = ctypes.c_int64(0)
    _check(h, load().pl_lognormal_prior(h, _ptr(pk), float(amp), _ptr(pk_log_out), ctypes.byref(mu),
                                        ctypes.byref(s0), ctypes.byref(nc)))
    return {"mu": mu.value, "sigma0_sq": s0.value, "n_clipped": int(nc.value)}


def pl_gaussian_map_solve(h, delta_inout, opts=None):
    info = pl_solve_info()
    rc = load().pl_gaussian_map_solve(h, _ptr(delta_inout), ctypes.byref(opts) if opts else None,
                                      ctypes.byref(info))
    _check(h, rc, allow=(PL_ERR_NOT_CONVERGED, PL_ERR_LINESEARCH))
    return info


def pl_linear_bias_grad(h, model, bk, x, grad_out, want_obj=True):
    obj = ctypes.c_double()
    _check(h, load().pl_linear_bias_grad(h, int(model), _ptr(bk), _ptr(x), _ptr(grad_out),
                                         ctypes.byref(obj) if want_obj else None))
    return obj.value if want_obj else None


def pl_linear_bias_hessvec(h, model, bk, x, v, hv_out):
    return _check(h, load().pl_linear_bias_hessvec(h, int(model), _ptr(bk), _ptr(x), _ptr(v), _ptr(hv_out)))


def pl_linear_bias_solve(h, model, bk, x_inout, opts=None):
    info = pl_solve_info()
    rc = load().pl_linear_bias_solve(h, int(model), _ptr(bk), _ptr(x_inout), ctypes.byref(opts) if opts else None,
                                     ctypes.byref(info))
    _check(h, rc, allow=(PL_ERR_NOT_CONVERGED, PL_ERR_LINESEARCH))
    return info


def pl_linear_bias_solve_hat(h, model, bk, x_inout, x_hat_out, opts=None):
    info = pl_solve_info()
    rc = load().pl_linear_bias_solve_hat(h, int(model), _ptr(bk), _ptr(x_inout), _ptr(x_hat_out),
                                         ctypes.byref(opts) if opts else None, ctypes.byref(info))
    _check(h, rc, allow=(PL_ERR_NOT_CONVERGED, PL_ERR_LINESEARCH))
    return info


def pl_nlcg_solve(h, s_inout, opts=None):
    info = pl_solve_info()
    rc = load().pl_nlcg_solve(h, _ptr(s_inout), ctypes.byref(opts) if opts else None, ctypes.byref(info))
    _check(h, rc, allow=(PL_ERR_NOT_CONVERGED, PL_ERR_LINESEARCH))
    return info


def pl_lsq_solve(h, delta_out, opts=None):
    info = pl_solve_info()
    rc = load().pl_lsq_solve(h, _ptr(delta_out), ctypes.byref(opts) if opts else None, ctypes.byref(info))
    _check(h, rc, allow=(PL_ERR_NOT_CONVERGED,))
    return info


def pl_inverse_weight(h, delta_out):
    return _check(h, load().pl_inverse_weight(h, _ptr(delta_out)))


def pl_compare_fields(h, rec, ref):
    r = ctypes.c_double(0.0)
    d = ctypes.c_double(0.0)
    _check(h, load().pl_compare_fields(h, _ptr(rec), _ptr(ref), ctypes.byref(r), ctypes.byref(d)))
    return r.value, d.value


def pl_compare_fields_noalloc(n, rec, ref, out, stream=None):
    """r and D_euc of rec against ref into the device tensor out (2 doubles),
    without a plan or workspace; asynchronous on `stream` (a hipStream_t
    handle, None for the default stream)."""
    nn = (ctypes.c_int32 * 3)(*[int(v) for v in n])
    rc = load().pl_compare_fields_noalloc(nn, _ptr(rec), _ptr(ref), _ptr(out), stream)
    if rc != PL_OK:
        raise PLError(rc, f"pl_compare_fields_noalloc(n={tuple(n)})")
    return rc


def pl_plan_prior_is_radial(h):
    out = ctypes.c_int32(0)
    _check(h, load().pl_plan_prior_is_radial(h, ctypes.byref(out)))
    return bool(out.value)


VARIANT_SLOTS = ("x_krylov", "y", "z", "x_operator", "table_krylov", "table_operator", "stream_nt")


def pl_plan_get_variants(h):
    """{precision: (x Krylov passes, y, z, x operator passes, table of the
    Krylov passes, table of the operator passes, streaming loads)}"""
    k = len(VARIANT_SLOTS)
    out = (ctypes.c_int32 * (2 * k))()
    _check(h, load().pl_plan_get_variants(h, out))
    return {"fp64": tuple(out[0:k]), "fp32": tuple(out[k:2 * k])}


def pl_plan_set_variants(h, fp64=(0, 0, 0, 0, 0, 0, 0), fp32=(0, 0, 0, 0, 1, 1, 0)):
    """Per precision, the choices in VARIANT_SLOTS order."""
    k = len(VARIANT_SLOTS)
    vals = tuple(int(x) for x in fp64) + tuple(int(x) for x in fp32)
    if len(vals) != 2 * k:
        raise ValueError(f"expected {k} choices per precision")
    v = (ctypes.c_int32 * (2 * k))(*vals)
    return _check(h, load().pl_plan_set_variants(h, v))


def pl_batch_create(ns, boxes, precision=PL_FP64, stream=None):
    """ns, boxes: sequences of 3-tuples.  Returns (handle, workspace_bytes)."""
    lib = load()
    k = len(ns)
    h = ctypes.c_void_p()
    nn = (ctypes.c_int32 * (3 * k))(*[int(v) for n in ns for v in n])
    bb = (ctypes.c_double * (3 * k))(*[float(v) for b in boxes for v in b])
    ws = ctypes.c_size_t()
    rc = lib.pl_batch_create(ctypes.byref(h), k, nn, bb, int(precision), stream, ctypes.byref(ws))
    if rc != PL_OK:
        raise PLError(rc, "pl_batch_create")
    return h, ws.value


def _bcheck(h, rc, allow=()):
    if rc != PL_OK and rc not in allow:
        raise PLError(rc, load().pl_batch_last_error(h).decode() if h else "")
    return rc


def pl_batch_set_workspace(h, ws_tensor):
    return _bcheck(h, load().pl_batch_set_workspace(h, _ptr(ws_tensor)))


def pl_batch_set_problem(h, i, w, counts, pk, amp, mu, nbar, beta=1.0, inv_p0=0.0):
    pr = pl_problem(_ptr(w).value, _ptr(counts).value, _ptr(pk).value, float(amp), float(mu), float(nbar),
                    float(beta), float(inv_p0))
    return _bcheck(h, load().pl_batch_set_problem(h, int(i), ctypes.byref(pr)))


def pl_batch_solve(h, s_list, opts=None):
    k = len(s_list)
    ptrs = (ctypes.c_void_p * k)(*[t.data_ptr() for t in s_list])
    infos = (pl_solve_info * k)()
    rc = load().pl_batch_solve(h, ptrs, ctypes.byref(opts) if opts else None, infos)
    _bcheck(h, rc, allow=(PL_ERR_NOT_CONVERGED, PL_ERR_LINESEARCH))
    return [infos[i].as_dict() for i in range(k)]


def pl_batch_autotune(h, cache_path=None):
    return _bcheck(h, load().pl_batch_autotune(h, cache_path.encode() if cache_path else None))


def pl_batch_destroy(h):
    return load().pl_batch_destroy(h)


def pl_batch_last_error(h):
    return load().pl_batch_last_error(h).decode()


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------

def make_opts(rtol=1e-8, max_newton=100, max_cg=500, eta_max=0.5, ls_c1=1e-4, precision=-1, check_every=8):
    o = pl_default_opts()
    o.rtol, o.max_newton, o.max_cg = float(rtol), int(max_newton), int(max_cg)
    o.eta_max, o.ls_c1, o.precision, o.check_every = float(eta_max), float(ls_c1), int(precision), int(check_every)
    return o


class Plan:
    """A grid + workspace on the current torch device and stream."""

    def __init__(self, n, box, precision="fp64", device="cuda", stream=None):
        import torch
        self.torch = torch
        self.n = tuple(int(v) for v in n)
        self.box = tuple(float(v) for v in box)
        self.device = torch.device(device)
        self.precision = PL_MIXED if precision in ("mixed", PL_MIXED) else PL_FP64
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = st
        self.h, ws_bytes = pl_plan_create(self.n, self.box, self.precision, ctypes.c_void_p(st.cuda_stream))
        self.ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self._ws_view = self.ws[off:]
        pl_plan_set_workspace(self.h, self._ws_view)
        self._keep = ()
        self.params = None  # set by set_problem

    @property
    def ncells(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def half_shape(self):
        return (self.n[0], self.n[1], self.n[2] // 2 + 1)

    def _dev(self, x, dtype=None):
        t = self.torch
        dtype = dtype or t.float64
        if isinstance(x, np.ndarray):
            x = t.from_numpy(np.ascontiguousarray(x))
        return x.to(device=self.device, dtype=dtype).contiguous()

    def set_problem(self, w, counts, pk, amp, mu, nbar, beta=1.0, inv_p0=0.0):
        w, counts, pk = self._dev(w), self._dev(counts), self._dev(pk)
        self._keep = (w, counts, pk)
        pl_set_problem(self.h, w, counts, pk, amp, mu, nbar, beta, inv_p0)
        self.params = dict(amp=amp, mu=mu, nbar=nbar, beta=beta, inv_p0=inv_p0)

    def set_instance(self, inst):
        self.set_problem(inst["w"], inst["counts"], inst["pk"], inst["amp"], inst["mu"], inst["nbar"],
                         inst.get("beta", 1.0), inst.get("inv_p0", 0.0))

    def grad(self, s, out=None):
        s = self._dev(s)
        out = self.torch.empty_like(s) if out is None else out
        obj = pl_grad(self.h, s, out)
        return out, obj

    def hessvec(self, v, s=None, out=None):
        v = self._dev(v)
        out = self.torch.empty_like(v) if out is None else out
        pl_hessvec(self.h, None if s is None else self._dev(s), v, out)
        return out

    def hessvec_f32(self, v, s=None, out=None):
        v = self._dev(v, self.torch.float32)
        out = self.torch.empty_like(v) if out is None else out
        pl_hessvec_f32(self.h, None if s is None else self._dev(s), v, out)
        return out

    def hessvec_hat(self, v_hat, out=None):
        out = self.torch.empty_like(v_hat) if out is None else out
        if v_hat.dtype == self.torch.complex128:
            pl_hessvec_hat(self.h, v_hat, out)
        else:
            pl_hessvec_hat_f32(self.h, v_hat, out)
        return out

    def solve(self, s0=None, want_hat=False, **kw):
        """MAP solve: (s, info), or (s, s_hat, info) with want_hat (the
        solver's half-spectrum iterate, complex128 on the device)."""
        if s0 is None:
            # s0 = mu (0 before a problem is set; the library then reports it)
            mu = float(self.params["mu"]) if self.params else 0.0
            s = self.torch.full(self.n, mu, dtype=self.torch.float64, device=self.device)
        else:
            s = self._dev(s0).clone()
        if want_hat:
            s_hat = self.torch.empty(self.half_shape, dtype=self.torch.complex128, device=self.device)
            info = pl_newton_krylov_solve_hat(self.h, s, s_hat, make_opts(**kw))
            return s, s_hat, info.as_dict()
        info = pl_newton_krylov_solve(self.h, s, make_opts(**kw))
        return s, info.as_dict()

    def adjoint(self, s_star, dL_ds, want_fields=True, **kw):
        s_star, dL_ds = self._dev(s_star), self._dev(dL_ds)
        lam = self.torch.empty_like(s_star)
        dN = self.torch.empty_like(s_star) if want_fields else None
        dw = self.torch.empty_like(s_star) if want_fields else None
        scal, info = pl_solve_adjoint(self.h, s_star, dL_ds, lam, dN, dw, make_opts(**kw))
        return dict(scal, N=dN, w=dw, lam=lam), info.as_dict()

    def solve_gaussian(self, delta0=None, **kw):
        """MAP overdensity of the Gaussian-prior model (eq. MAPG): (delta, info)."""
        if delta0 is None:
            d = self.torch.zeros(self.n, dtype=self.torch.float64, device=self.device)
        else:
            d = self._dev(delta0).clone()
        info = pl_gaussian_map_solve(self.h, d, make_opts(**kw))
        return d, info.as_dict()

    def _model(self, model):
        return MODELS[model] if isinstance(model, str) else int(model)

    def linear_bias_grad(self, model, bk, x, out=None):
        """Gradient and objective of the linear-bias posterior at x (sections
        2.2.1 / 2.4.1); model "lognormal" (x = s) or "gaussian" (x = delta)."""
        x, bk = self._dev(x), self._dev(bk)
        out = self.torch.empty_like(x) if out is None else out
        obj = pl_linear_bias_grad(self.h, self._model(model), bk, x, out)
        return out, obj

    def linear_bias_hessvec(self, model, bk, v, x=None, out=None):
        v, bk = self._dev(v), self._dev(bk)
        out = self.torch.empty_like(v) if out is None else out
        pl_linear_bias_hessvec(self.h, self._model(model), bk, None if x is None else self._dev(x), v, out)
        return out

    def solve_linear_bias(self, model, bk, x0=None, want_hat=False, **kw):
        """MAP with the linear bias b_hat (bk, half spectrum): (x, info); the
        start defaults to the prior mean (mu, or 0 for the Gaussian prior)."""
        m = self._model(model)
        bk = self._dev(bk)
        if x0 is None:
            mu = float(self.params["mu"]) if (self.params and m == MODEL_LOGNORMAL) else 0.0
            x = self.torch.full(self.n, mu, dtype=self.torch.float64, device=self.device)
        else:
            x = self._dev(x0).clone()
        kw.setdefault("precision", 0)
        if want_hat:
            x_hat = self.torch.empty(self.half_shape, dtype=self.torch.complex128, device=self.device)
            info = pl_linear_bias_solve_hat(self.h, m, bk, x, x_hat, make_opts(**kw))
            return x, x_hat, info.as_dict()
        info = pl_linear_bias_solve(self.h, m, bk, x, make_opts(**kw))
        return x, info.as_dict()

    def solve_nlcg(self, s0=None, **kw):
        """MAP by the Krylov step with nonlinear-CG search vectors (FP64)."""
        if s0 is None:
            # s0 = mu (0 before a problem is set; the library then reports it)
            mu = float(self.params["mu"]) if self.params else 0.0
            s = self.torch.full(self.n, mu, dtype=self.torch.float64, device=self.device)
        else:
            s = self._dev(s0).clone()
        kw.setdefault("precision", 0)
        info = pl_nlcg_solve(self.h, s, make_opts(**kw))
        return s, info.as_dict()

    def lognormal_prior(self, pk, amp):
        """Log-field spectrum P_L (device, half spectrum, for amp = 1) and
        {mu, sigma0_sq, n_clipped} from the matter spectrum amp * pk."""
        out = self.torch.empty(self.half_shape, dtype=self.torch.float64, device=self.device)
        info = pl_lognormal_prior(self.h, self._dev(pk), amp, out)
        return out, info

    def lsq(self, **kw):
        """LSQ-Wiener overdensity of the current problem: (delta, info)."""
        delta = self.torch.empty(self.n, dtype=self.torch.float64, device=self.device)
        info = pl_lsq_solve(self.h, delta, make_opts(**kw))
        return delta, info.as_dict()

    def inverse_weight(self):
        """Inverse-weighted overdensity N / (w nbar) - 1 (0 where w = 0)."""
        delta = self.torch.empty(self.n, dtype=self.torch.float64, device=self.device)
        pl_inverse_weight(self.h, delta)
        return delta

    def compare(self, rec, ref):
        """(correlation coefficient, Euclidean distance) of rec against ref."""
        return pl_compare_fields(self.h, self._dev(rec), self._dev(ref))

    def autotune(self, cache_path=None):
        """Pick the fastest tile variants for this grid (needs set_problem)."""
        pl_plan_autotune(self.h, cache_path)
        return pl_plan_get_variants(self.h)

    def close(self):
        if self.h:
            pl_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent reconstructions solved together (one launch per pass)."""

    def __init__(self, instances, precision="mixed", device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.precision = PL_MIXED if precision in ("mixed", PL_MIXED) else PL_FP64
        self.ns = [tuple(int(v) for v in it["n"]) for it in instances]
        boxes = [tuple(float(v) for v in it["box"]) for it in instances]
        st = torch.cuda.current_stream(self.device)
        self.h, ws_bytes = pl_batch_create(self.ns, boxes, self.precision, ctypes.c_void_p(st.cuda_stream))
        self.ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        pl_batch_set_workspace(self.h, self.ws[off:])
        self._keep = []
        self.mus = []
        for i, it in enumerate(instances):
            w, c, pk = (torch.from_numpy(np.ascontiguousarray(it[k])).to(self.device, torch.float64)
                        for k in ("w", "counts", "pk"))
            self._keep.append((w, c, pk))
            pl_batch_set_problem(self.h, i, w, c, pk, it["amp"], it["mu"], it["nbar"], it.get("beta", 1.0),
                                 it.get("inv_p0", 0.0))
            self.mus.append(float(it["mu"]))

    def autotune(self, cache_path=None):
        """Pick the batched passes' tile variants per grid length (by timing,
        or from cache_path)."""
        pl_batch_autotune(self.h, cache_path)

    def solve(self, s0_list=None, **kw):
        t = self.torch
        if s0_list is None:
            s = [t.full(n, mu, dtype=t.float64, device=self.device) for n, mu in zip(self.ns, self.mus)]
        else:
            s = [x.to(self.device, t.float64).clone() for x in s0_list]
        infos = pl_batch_solve(self.h, s, make_opts(**kw))
        return s, infos

    def close(self):
        if self.h:
            pl_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
