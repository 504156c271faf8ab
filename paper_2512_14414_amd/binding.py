"""ctypes binding of libctm.so (include/ctm.h).

Argument marshalling only: torch tensors provide device memory and the
stream; every step of the computation runs in the library's HIP kernels.
There is no fallback: if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctm.so")

CTM_OK, CTM_ENOTCONV = 0, 1
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "mixed": 3}


class CTMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ctm error {code}: {msg}")
        self.code = code


class Term(ctypes.Structure):
    _fields_ = [("px", ctypes.c_int), ("py", ctypes.c_int), ("a", ctypes.c_int), ("b", ctypes.c_int),
                ("coef", ctypes.c_double)]


# ctm_alloc_fn / ctm_free_fn of include/ctm.h
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2512_14414_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    sig = {
        "ctm_init": (I, [ctypes.POINTER(P), P, I, I, I, I, I, ctypes.POINTER(I), I, I, P]),
        "ctm_init_double_layer": (I, [ctypes.POINTER(P), P, I, I, I, I, I, ctypes.POINTER(I), I, I, P]),
        "ctm_set_tensors": (I, [P, P]),
        "ctm_reset_env": (I, [P]),
        "ctm_env_size": (I64, [P]),
        "ctm_set_env": (I, [P, P]),
        "ctm_get_env": (I, [P, P]),
        "ctm_sweep": (I, [P, I, D, ctypes.POINTER(I), ctypes.POINTER(D)]),
        "ctm_energy": (I, [P, ctypes.POINTER(D), I, ctypes.POINTER(Term), ctypes.POINTER(D)]),
        "ctm_energy_grad": (I, [P, P, I, ctypes.POINTER(D), I, ctypes.POINTER(Term), ctypes.POINTER(D), P]),
        "ctm_energy_grad_fp": (I, [P, P, D, I, ctypes.POINTER(D), I, ctypes.POINTER(Term), ctypes.POINTER(D), P,
                                   ctypes.POINTER(I), ctypes.POINTER(D)]),
        "ctm_last_rdms": (I, [P, ctypes.POINTER(D), I, ctypes.POINTER(I)]),
        "ctm_observables": (I, [P, ctypes.POINTER(D), I, ctypes.POINTER(I)]),
        "ctm_corner_spectra": (I, [P, ctypes.POINTER(D), I64, ctypes.POINTER(I64)]),
        "ctm_set_option": (I, [P, ctypes.c_char_p, D]),
        "ctm_set_allocator": (I, [P, ALLOC_FN, FREE_FN, P]),
        "ctm_profile_begin": (I, [P]),
        "ctm_profile_end": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I64)]),
        "ctm_last_error": (ctypes.c_char_p, [P]),
        "ctm_free": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    return lib


LIB = _load()
EXPORTED = ("ctm_init", "ctm_init_double_layer", "ctm_set_tensors", "ctm_reset_env", "ctm_env_size", "ctm_set_env", "ctm_get_env",
            "ctm_sweep", "ctm_corner_spectra", "ctm_energy", "ctm_energy_grad", "ctm_energy_grad_fp", "ctm_last_rdms",
            "ctm_observables",
            "ctm_set_option", "ctm_set_allocator", "ctm_profile_begin", "ctm_profile_end",
            "ctm_last_error", "ctm_free")


def _terms(terms):
    arr = (Term * max(1, len(terms)))()
    for i, (px, py, a, b, coef) in enumerate(terms):
        arr[i] = Term(px, py, a, b, coef)
    return arr


def _hbond(H):
    vals = torch.as_tensor(H, dtype=torch.float64).reshape(-1).tolist()
    return (ctypes.c_double * len(vals))(*[float(v) for v in vals])


def torch_allocator(device=None):
    """(alloc, free) for CTM.set_allocator backed by PyTorch's caching allocator:
    alloc(nbytes, stream) -> device pointer (0 when it has no memory),
    free(ptr, stream)."""
    dev = torch.cuda.current_device() if device is None else device

    def alloc(nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(nbytes, device=dev, stream=stream)
        except RuntimeError:
            return 0

    def free(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


def _dptr(t: torch.Tensor, dtype=torch.float64):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("expected a contiguous CUDA tensor of dtype %s" % dtype)
    return ctypes.c_void_p(t.data_ptr())


class CTM:
    """A CTMRG context on the current GPU (one per set of site tensors).

    layout "nested" (ctm_init): the single-layer nested network; "double"
    (ctm_init_double_layer): the double-layer network of reduced tensors."""

    def __init__(self, A, pattern, chi, precision="fp64", stream=None, layout="nested"):
        A = torch.as_tensor(A, dtype=torch.float64)
        if not A.is_cuda:
            A = A.cuda()
        self.A = A.contiguous()
        n_t, d, D = self.A.shape[0], self.A.shape[1], self.A.shape[2]
        self.d, self.D, self.chi = d, D, chi
        self.Ly, self.Lx = len(pattern), len(pattern[0])
        self.pattern = pattern
        flat = (ctypes.c_int * (self.Lx * self.Ly))(*[pattern[y][x] for y in range(self.Ly) for x in range(self.Lx)])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = ctypes.c_void_p()
        init = {"nested": LIB.ctm_init, "double": LIB.ctm_init_double_layer}[layout]
        self.layout = layout
        rc = init(ctypes.byref(self._h), _dptr(self.A), d, D, chi, self.Lx, self.Ly, flat, n_t,
                  PRECISIONS[precision], ctypes.c_void_p(self.stream.cuda_stream))
        if rc != CTM_OK:
            raise CTMError(rc, LIB.ctm_last_error(None).decode())

    def _check(self, rc, allow=(CTM_OK,)):
        if rc not in allow:
            raise CTMError(rc, LIB.ctm_last_error(self._h).decode())
        return rc

    def close(self):
        if self._h:
            LIB.ctm_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_allocator(self, alloc=None, free=None):
        """ctm_set_allocator: new device blocks of the context from alloc(nbytes,
        stream) -> pointer (0 for none) and back through free(ptr, stream), with
        stream the integer hipStream_t of the context's stream that uses the
        block; torch_allocator() gives PyTorch's caching allocator.  No
        arguments restore the default for new blocks."""
        if (alloc is None) != (free is None):
            raise ValueError("alloc and free must both be given or both be None")
        if alloc is None:
            cbs = (ALLOC_FN(), FREE_FN())
        else:
            cbs = (ALLOC_FN(lambda n, st, u: alloc(int(n), st or 0) or None),
                   FREE_FN(lambda ptr, st, u: free(ptr, st or 0)))
        self._check(LIB.ctm_set_allocator(self._h, cbs[0], cbs[1], None))
        # every pair stays referenced as long as the object: blocks are handed
        # back through the callbacks that made them, inside ctm_free at the latest
        self._alloc_keep = getattr(self, "_alloc_keep", []) + [cbs]

    def set_tensors(self, A):
        self.A = torch.as_tensor(A, dtype=torch.float64).cuda().contiguous()
        self._check(LIB.ctm_set_tensors(self._h, _dptr(self.A)))

    def reset_env(self):
        self._check(LIB.ctm_reset_env(self._h))

    def env_size(self):
        return int(LIB.ctm_env_size(self._h))

    def get_env(self):
        out = torch.empty(self.env_size(), dtype=torch.float64, device=self.A.device)
        self._check(LIB.ctm_get_env(self._h, _dptr(out)))
        return out

    def set_env(self, env):
        env = torch.as_tensor(env, dtype=torch.float64).to(self.A.device).contiguous()
        if env.numel() != self.env_size():
            raise ValueError("environment has the wrong size")
        self._check(LIB.ctm_set_env(self._h, _dptr(env)))

    def sweep(self, max_sweeps, tol=0.0):
        n, dl = ctypes.c_int(), ctypes.c_double()
        rc = self._check(LIB.ctm_sweep(self._h, max_sweeps, tol, ctypes.byref(n), ctypes.byref(dl)),
                         allow=(CTM_OK, CTM_ENOTCONV))
        return n.value, dl.value, rc == CTM_OK

    def energy(self, H, terms):
        E = ctypes.c_double()
        self._check(LIB.ctm_energy(self._h, _hbond(H), len(terms), _terms(terms), ctypes.byref(E)))
        return E.value

    def energy_grad(self, n_sweeps, H, terms, A=None):
        """(E, dE/dA) after ``n_sweeps`` sweeps from the current environment (held constant).

        If A is given it replaces the site tensors first.  The environment is
        left at the result of the sweeps."""
        aptr = None
        if A is not None:
            self.A = torch.as_tensor(A, dtype=torch.float64).to(self.A.device).contiguous()
            aptr = _dptr(self.A)
        g = torch.empty_like(self.A)
        E = ctypes.c_double()
        self._check(LIB.ctm_energy_grad(self._h, aptr, int(n_sweeps), _hbond(H), len(terms), _terms(terms),
                                        ctypes.byref(E), _dptr(g)))
        return E.value, g

    def energy_grad_fp(self, H, terms, tol=1e-12, max_iter=500, A=None):
        """(E, dE/dA, terms of the series, fixed-point gap, converged) of the converged energy
        (ctm_energy_grad_fp); the current environment must be converged."""
        aptr = None
        if A is not None:
            self.A = torch.as_tensor(A, dtype=torch.float64).to(self.A.device).contiguous()
            aptr = _dptr(self.A)
        g = torch.empty_like(self.A)
        E, it, gap = ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
        rc = self._check(LIB.ctm_energy_grad_fp(self._h, aptr, tol, max_iter, _hbond(H), len(terms), _terms(terms),
                                                ctypes.byref(E), _dptr(g), ctypes.byref(it), ctypes.byref(gap)),
                         allow=(CTM_OK, CTM_ENOTCONV))
        return E.value, g, it.value, gap.value, rc == CTM_OK

    def last_rdms(self, capacity=16):
        d8 = self.d ** 8
        buf = (ctypes.c_double * (capacity * d8))()
        n = ctypes.c_int()
        self._check(LIB.ctm_last_rdms(self._h, buf, capacity, ctypes.byref(n)))
        k = min(n.value, capacity)
        d4 = self.d ** 4
        return torch.tensor(list(buf[: k * d8]), dtype=torch.float64).reshape(k, d4, d4)

    def corner_spectra(self):
        """Normalised corner spectra (ctm_corner_spectra): rows = nested positions row-major x (C1..C4), chi each."""
        n = ctypes.c_int64()
        self._check(LIB.ctm_corner_spectra(self._h, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_double * n.value)()
        self._check(LIB.ctm_corner_spectra(self._h, buf, n.value, ctypes.byref(n)))
        return torch.tensor(list(buf), dtype=torch.float64).reshape(-1, self.chi)

    N_OBS = 18   # CTM_N_OBS of include/ctm.h

    def observables(self, capacity=16):
        """Per plaquette of the last energy call: the (x, y, z) moments of TL, TR, BL, BR, then the six
        bond correlations (ctm_observables)."""
        buf = (ctypes.c_double * (capacity * self.N_OBS))()
        n = ctypes.c_int()
        self._check(LIB.ctm_observables(self._h, buf, capacity, ctypes.byref(n)))
        k = min(n.value, capacity)
        return torch.tensor(list(buf[: k * self.N_OBS]), dtype=torch.float64).reshape(k, self.N_OBS)

    def profile_begin(self):
        self._check(LIB.ctm_profile_begin(self._h))

    FAMILIES = ("fp64", "fp32", "bf16", "jacobi", "qr_panel")

    def profile_end(self):
        """{family: (kernel ms, algorithmic flops, launches)} for the contraction
        kernel on the fp64, fp32 and bf16 paths, the block Jacobi rounds and the QR panels."""
        n_f = len(self.FAMILIES)
        ms, fl, n = (ctypes.c_double * n_f)(), (ctypes.c_double * n_f)(), (ctypes.c_int64 * n_f)()
        self._check(LIB.ctm_profile_end(self._h, ms, fl, n))
        return {k: (ms[i], fl[i], n[i]) for i, k in enumerate(self.FAMILIES)}

    def set_option(self, key, value):
        self._check(LIB.ctm_set_option(self._h, key.encode(), float(value)))


# ---------------------------------------------------------------------------
# Optimisation layer (include/ctm_opt.h)

class LBFGSParams(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("history", ctypes.c_int), ("c1", ctypes.c_double),
                ("c2", ctypes.c_double), ("gtol", ctypes.c_double), ("max_ls", ctypes.c_int),
                ("alpha0", ctypes.c_double), ("sur_start", ctypes.c_int), ("n_trials", ctypes.c_int),
                ("max_screened", ctypes.c_int), ("refit_every", ctypes.c_int), ("refit_steps", ctypes.c_int),
                ("lr", ctypes.c_float), ("n_blocks", ctypes.c_int), ("extrap", ctypes.c_int),
                ("window", ctypes.c_int)]


class LBFGSRecord(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int), ("evals", ctypes.c_int), ("screened", ctypes.c_int), ("f", ctypes.c_double),
                ("gmax", ctypes.c_double), ("step", ctypes.c_double)]


class EnergyObjective(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("H_bond", ctypes.POINTER(ctypes.c_double)), ("n_terms", ctypes.c_int),
                ("terms", ctypes.POINTER(Term)), ("conv_sweeps", ctypes.c_int), ("conv_tol", ctypes.c_double),
                ("grad_sweeps", ctypes.c_int)]


OBJECTIVE = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                             ctypes.c_void_p)


def _load_opt():
    P, I, I64, F = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
    sig = {
        "sur_init": (I, [ctypes.POINTER(P), I, I, ctypes.c_uint64, P]),
        "sur_param_count": (I64, [P]),
        "sur_get_params": (I, [P, P]),
        "sur_set_params": (I, [P, P]),
        "sur_predict": (I, [P, P, I, P]),
        "sur_predict_noalloc": (I, [P, P, I, P]),
        "sur_loss_grad": (I, [P, P, P, I, ctypes.POINTER(F), P]),
        "sur_train": (I, [P, P, P, I, I, F, ctypes.POINTER(F)]),
        "sur_last_error": (ctypes.c_char_p, [P]),
        "sur_free": (None, [P]),
        "ctm_lbfgs_default_params": (None, [ctypes.POINTER(LBFGSParams)]),
        "ctm_lbfgs": (I, [I64, P, OBJECTIVE, P, P, ctypes.POINTER(LBFGSParams), P, ctypes.POINTER(LBFGSRecord), I,
                          ctypes.POINTER(I)]),
        "ctm_lbfgs_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(LIB, name)
        f.restype, f.argtypes = res, args


_load_opt()
_HIP = ctypes.CDLL("libamdhip64.so")
_HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
_HIP.hipMemcpy.restype = ctypes.c_int


def _d2d(dst, src, nbytes):
    """Synchronous device-to-device copy between raw device addresses."""
    torch.cuda.synchronize()
    rc = _HIP.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


def _fptr(t: torch.Tensor):
    return _dptr(t, torch.float32)


class Surrogate:
    """The energy surrogate network on the current GPU (include/ctm_opt.h)."""

    def __init__(self, n_in, width=256, seed=0, stream=None):
        self.n_in, self.width = n_in, width
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = ctypes.c_void_p()
        rc = LIB.sur_init(ctypes.byref(self._h), n_in, width, seed, ctypes.c_void_p(self.stream.cuda_stream))
        if rc != CTM_OK:
            raise CTMError(rc, LIB.sur_last_error(None).decode())

    def _check(self, rc):
        if rc != CTM_OK:
            raise CTMError(rc, LIB.sur_last_error(self._h).decode())

    def close(self):
        if self._h:
            LIB.sur_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def param_count(self):
        return int(LIB.sur_param_count(self._h))

    def get_params(self):
        out = torch.empty(self.param_count(), dtype=torch.float32, device="cuda")
        self._check(LIB.sur_get_params(self._h, _fptr(out)))
        return out

    def set_params(self, theta):
        theta = torch.as_tensor(theta, dtype=torch.float32).cuda().contiguous()
        self._check(LIB.sur_set_params(self._h, _fptr(theta)))
        torch.cuda.synchronize()

    def predict(self, X):
        X = torch.as_tensor(X, dtype=torch.float32).cuda().contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        self._check(LIB.sur_predict(self._h, _fptr(X), X.shape[0], _fptr(y)))
        torch.cuda.synchronize()
        return y

    def predict_noalloc(self, X):
        """sur_predict_noalloc: the prediction with every workspace in the library's fixed scratch array."""
        X = torch.as_tensor(X, dtype=torch.float32).cuda().contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        self._check(LIB.sur_predict_noalloc(self._h, _fptr(X), X.shape[0], _fptr(y)))
        torch.cuda.synchronize()
        return y

    def loss_grad(self, X, t):
        X = torch.as_tensor(X, dtype=torch.float32).cuda().contiguous()
        t = torch.as_tensor(t, dtype=torch.float32).cuda().contiguous()
        g = torch.empty(self.param_count(), dtype=torch.float32, device="cuda")
        loss = ctypes.c_float()
        self._check(LIB.sur_loss_grad(self._h, _fptr(X), _fptr(t), X.shape[0], ctypes.byref(loss), _fptr(g)))
        return loss.value, g

    def train(self, X, t, steps, lr=1e-3):
        X = torch.as_tensor(X, dtype=torch.float32).cuda().contiguous()
        t = torch.as_tensor(t, dtype=torch.float32).cuda().contiguous()
        loss = ctypes.c_float()
        self._check(LIB.sur_train(self._h, _fptr(X), _fptr(t), X.shape[0], steps, lr, ctypes.byref(loss)))
        return loss.value


def lbfgs_params(**kw):
    p = LBFGSParams()
    LIB.ctm_lbfgs_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def python_objective(fn, n):
    """Wrap fn(x: cuda float64 tensor) -> (f, g) as a C objective (used by tests)."""
    def cb(user, xp, fp, gp):
        try:
            x = torch.empty(n, dtype=torch.float64, device="cuda")
            _d2d(x.data_ptr(), xp, n * 8)
            f, g = fn(x)
            g = torch.as_tensor(g, dtype=torch.float64, device="cuda").contiguous()
            fp[0] = float(f)
            _d2d(gp, g.data_ptr(), n * 8)
            return 0
        except Exception:
            import traceback
            traceback.print_exc()
            return -1
    return OBJECTIVE(cb)


def lbfgs(x0, objective, user=None, sur=None, params=None, capacity=10000):
    """Run ctm_lbfgs from x0 (float64 tensor); objective is an OBJECTIVE (see
    python_objective) or an EnergyObjective.  Returns (x, records, converged)."""
    x = torch.as_tensor(x0, dtype=torch.float64).cuda().contiguous().clone()
    params = params if params is not None else lbfgs_params()
    if isinstance(objective, EnergyObjective):
        fn = ctypes.cast(LIB.ctm_energy_objective_fn, OBJECTIVE)
        user = ctypes.cast(ctypes.pointer(objective), ctypes.c_void_p)
    else:
        fn = objective
    trace = (LBFGSRecord * capacity)()
    n_iter = ctypes.c_int()
    stream = torch.cuda.current_stream()
    rc = LIB.ctm_lbfgs(x.numel(), _dptr(x), fn, user, sur.handle if sur is not None else None, ctypes.byref(params),
                       ctypes.c_void_p(stream.cuda_stream), trace, capacity, ctypes.byref(n_iter))
    if rc not in (CTM_OK, CTM_ENOTCONV):
        raise CTMError(rc, LIB.ctm_lbfgs_last_error().decode())
    recs = [(r.iter, r.evals, r.screened, r.f, r.gmax, r.step) for r in trace[: min(n_iter.value, capacity)]]
    return x, recs, rc == CTM_OK


def energy_objective(ctm, H, terms, conv_sweeps=20, conv_tol=1e-9, grad_sweeps=1):
    """The library's energy objective over a CTM context (keeps its arrays alive)."""
    ob = EnergyObjective()
    ob._H = _hbond(H)
    ob._terms = _terms(terms)
    ob.ctx = ctm._h
    ob.H_bond = ctypes.cast(ob._H, ctypes.POINTER(ctypes.c_double))
    ob.n_terms = len(terms)
    ob.terms = ctypes.cast(ob._terms, ctypes.POINTER(Term))
    ob.conv_sweeps = conv_sweeps
    ob.conv_tol = conv_tol
    ob.grad_sweeps = grad_sweeps
    return ob
