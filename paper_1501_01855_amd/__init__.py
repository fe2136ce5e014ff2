"""MI355X (gfx950) overlap-operator library: Python binding of the C ABI.

Argument marshalling only: every step runs in the HIP library ``libovl.so``
built from ``csrc/``.  Fields are torch complex128 tensors on the GPU in the
canonical layout (``psi[..., V, 4, 3]``, ``U[V, 4, 3, 3]``, site
lexicographic with x fastest).  The library must be built
(``python -m paper_1501_01855_amd.build``); importing this module on a
machine without it raises immediately -- there is no fallback path.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libovl.so")

F64, F32, HALF = 0, 1, 2
SRC_POINT, SRC_GAUSS, SRC_Z2 = 0, 1, 2
MAX_NZ = 64
KERN_STENCIL, KERN_SHIFT = 0, 1
N_STENCIL_VARIANTS = 22   # launch variants of the stencil (tuning-table values 0 .. 21)
OPT_GRAPHS, OPT_AUTOTUNE, OPT_ADAPTIVE_NZ, OPT_BOUND_PRINTED, OPT_TWO_ROW_LINKS, OPT_OUTER_PRINTED = 1, 2, 3, 4, 5, 6

STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_HIP", -3: "ERR_NOMEM", -4: "ERR_NOT_CONVERGED",
          -5: "ERR_BREAKDOWN", -6: "ERR_UNSUPPORTED", -7: "ERR_STATE"}


class OvlError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Zolo(ctypes.Structure):
    _fields_ = [("n_z", ctypes.c_int32), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("delta", ctypes.c_double), ("omega", ctypes.c_double * MAX_NZ),
                ("sigma", ctypes.c_double * MAX_NZ)]

    @property
    def omegas(self):
        return [self.omega[i] for i in range(self.n_z)]

    @property
    def sigmas(self):
        return [self.sigma[i] for i in range(self.n_z)]


class Stats(ctypes.Structure):
    _fields_ = [("dslash_calls", ctypes.c_int64 * 3), ("sign_calls", ctypes.c_int64 * 3),
                ("mscg_iters", ctypes.c_int64), ("sumr_iters", ctypes.c_int64),
                ("gmresr_steps", ctypes.c_int64), ("restarts", ctypes.c_int64),
                ("computed_relres", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {"dslash_calls": list(self.dslash_calls), "sign_calls": list(self.sign_calls),
                "mscg_iters": self.mscg_iters, "sumr_iters": self.sumr_iters,
                "gmresr_steps": self.gmresr_steps, "restarts": self.restarts,
                "computed_relres": self.computed_relres, "seconds": self.seconds,
                # the paper's cost unit: a double-precision Wilson call counts 2, single 1
                "wilson_units": 2 * self.dslash_calls[0] + self.dslash_calls[1] + self.dslash_calls[2]}


class SolverParams(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("mu", ctypes.c_double), ("tol", ctypes.c_double),
                ("eta_tilde", ctypes.c_double), ("relax_floor", ctypes.c_double),
                ("f32_threshold", ctypes.c_double), ("half_threshold", ctypes.c_double),
                ("norm_restart", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("max_middle", ctypes.c_int32), ("max_mscg", ctypes.c_int32),
                ("use_deflation", ctypes.c_int32), ("eig_calc", ctypes.c_int32),
                ("n_eig", ctypes.c_int32), ("m_eig", ctypes.c_int32), ("k_recalc", ctypes.c_int32),
                ("verbose", ctypes.c_int32), ("eig_eps", ctypes.c_double),
                ("delta_split", ctypes.c_double), ("middle_cg", ctypes.c_int32),
                ("eig_block", ctypes.c_int32)]


EXPORTS = ["ovl_create", "ovl_destroy", "ovl_last_error", "ovl_solver_defaults", "ovl_device_bytes",
           "ovl_gauge_load", "ovl_gauge_generate", "ovl_source_generate", "ovl_wilson_dslash",
           "ovl_kernel_K_apply", "ovl_zolotarev_coeffs", "ovl_lowmodes_compute", "ovl_lowmodes_set",
           "ovl_lowmodes_get", "ovl_sign_zolotarev_mscg", "ovl_overlap_apply",
           "ovl_sumr_gmresr_solve", "ovl_profile_enable", "ovl_profile_read", "ovl_eigspace_info",
           "ovl_eigspace_get", "ovl_eigspace_set", "ovl_eigspace_diagonalise", "ovl_eigspace_recompute",
           "ovl_deflate_project", "ovl_overlap_adjoint", "ovl_tuning_get", "ovl_tuning_set", "ovl_set_option",
           "ovl_sumr_gmresr_solve_many", "ovl_eigsumr_eigensolve", "ovl_wilson_dslash_noalloc",
           "ovl_kernel_interval", "ovl_stream_bench", "ovl_eigspace_save", "ovl_eigspace_load",
           "ovl_sign_lanczos", "ovl_gauge_info"]

_lib = None


def lib():
    """Load libovl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1501_01855_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "ovl_create": ([P, P, P], I32),
        "ovl_destroy": ([P], I32),
        "ovl_last_error": ([], ctypes.c_char_p),
        "ovl_solver_defaults": ([P], None),
        "ovl_device_bytes": ([P], I64),
        "ovl_gauge_load": ([P, P], I32),
        "ovl_gauge_generate": ([P, ctypes.c_uint64, D, P], I32),
        "ovl_source_generate": ([P, I32, ctypes.c_uint64, I64, I32, I32, P], I32),
        "ovl_wilson_dslash": ([P, P, P, I32, I32], I32),
        "ovl_wilson_dslash_noalloc": ([P, P, P, I32, I32], I32),
        "ovl_kernel_K_apply": ([P, D, P, P, I32, I32], I32),
        "ovl_zolotarev_coeffs": ([I32, D, D, P], I32),
        "ovl_lowmodes_compute": ([P, D, I32, D, P, P], I32),
        "ovl_lowmodes_set": ([P, I32, P, P], I32),
        "ovl_kernel_interval": ([P, D, I32, P, P, P], I32),
        "ovl_lowmodes_get": ([P, P], I32),
        "ovl_sign_zolotarev_mscg": ([P, D, P, P, P, I32, D, I32, P], I32),
        "ovl_overlap_apply": ([P, D, D, P, P, P, I32, D, I32, P], I32),
        "ovl_sign_lanczos": ([P, D, P, P, P, I32, D, P], I32),
        "ovl_overlap_adjoint": ([P, D, D, P, P, P, I32, D, I32, P, P, P], I32),
        "ovl_tuning_get": ([P, P, P, I32, P], I32),
        "ovl_tuning_set": ([P, P, P, I32], I32),
        "ovl_set_option": ([P, I32, I32], I32),
        "ovl_gauge_info": ([P, P, P], I32),
        "ovl_stream_bench": ([P, I32, P, P, I64, I32, P], I32),
        "ovl_sumr_gmresr_solve_many": ([P, I32, P], I32),
        "ovl_sumr_gmresr_solve": ([P, P, P, P, P, I32, P], I32),
        "ovl_profile_enable": ([P, I32], I32),
        "ovl_profile_read": ([P, I32, I32, P, P, P], I32),
        "ovl_eigspace_info": ([P, P, I32, P, P, P], I32),
        "ovl_eigspace_get": ([P, P, P], I32),
        "ovl_eigspace_set": ([P, I32, I32, D, D, I32, P, P], I32),
        "ovl_eigspace_diagonalise": ([P], I32),
        "ovl_eigspace_save": ([P, ctypes.c_char_p], I32),
        "ovl_eigspace_load": ([P, ctypes.c_char_p], I32),
        "ovl_eigspace_recompute": ([P, D, P, D], I32),
        "ovl_deflate_project": ([P, P, P, P, I32], I32),
        "ovl_eigsumr_eigensolve": ([P, P, P, P, I32, I32, D, P, P, P, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(code, allow=()):
    if code != 0 and code not in allow:
        msg = lib().ovl_last_error()
        raise OvlError(code, msg.decode() if msg else "")
    return code


def _dev(t, shape_tail, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.complex128:
        raise TypeError(f"{name}: expected a complex128 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name}: trailing shape {tuple(t.shape)} does not end with {shape_tail}")
    return ctypes.c_void_p(t.data_ptr())


def zolotarev_coeffs(n_z, a, b):
    z = Zolo()
    _check(lib().ovl_zolotarev_coeffs(int(n_z), float(a), float(b), ctypes.byref(z)))
    return z


def zolo_from(n_z, a, b, delta, omega, sigma):
    """Build coefficients from given data (e.g. shared with a reference)."""
    z = Zolo()
    z.n_z, z.a, z.b, z.delta = int(n_z), float(a), float(b), float(delta)
    for i in range(int(n_z)):
        z.omega[i] = float(omega[i])
        z.sigma[i] = float(sigma[i])
    return z


def solver_defaults(**kw):
    p = SolverParams()
    lib().ovl_solver_defaults(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


class Context:
    """One lattice (extents dims = (Lx, Ly, Lz, Lt)) on the current GPU."""

    def __init__(self, dims, stream=None):
        self.dims = tuple(int(d) for d in dims)
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        d = (ctypes.c_int32 * 4)(*self.dims)
        _check(lib().ovl_create(d, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ovl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device_bytes(self):
        return lib().ovl_device_bytes(self._h)

    # -- inputs
    def gauge_load(self, U):
        _check(lib().ovl_gauge_load(self._h, _dev(U, (self.V, 4, 3, 3), "U")))

    def gauge_generate(self, seed, eps, out=None):
        p = _dev(out, (self.V, 4, 3, 3), "out") if out is not None else None
        _check(lib().ovl_gauge_generate(self._h, int(seed), float(eps), p))
        return out

    def source(self, kind, seed=0, site=0, spin=0, colour=0):
        out = torch.empty((self.V, 4, 3), dtype=torch.complex128, device="cuda")
        _check(lib().ovl_source_generate(self._h, int(kind), int(seed), int(site), int(spin),
                                         int(colour), _dev(out, (self.V, 4, 3), "out")))
        return out

    # -- operators
    def _nrhs(self, psi):
        return 1 if psi.dim() == 3 else int(psi.shape[0])

    def wilson_dslash(self, psi, prec=F64):
        out = torch.empty_like(psi)
        _check(lib().ovl_wilson_dslash(self._h, _dev(psi, (self.V, 4, 3), "psi"),
                                       _dev(out, (self.V, 4, 3), "out"), self._nrhs(psi), prec))
        return out

    def wilson_dslash_noalloc(self, psi, out, prec=F64):
        """H psi into the caller's out, with no device allocation by the library
        (packed copies in its fixed scratch array); returns the status."""
        return _check(lib().ovl_wilson_dslash_noalloc(self._h, _dev(psi, (self.V, 4, 3), "psi"),
                                                      _dev(out, (self.V, 4, 3), "out"), self._nrhs(psi), prec),
                      allow=(-1,))

    def kernel_K_apply(self, psi, rho, prec=F64):
        out = torch.empty_like(psi)
        _check(lib().ovl_kernel_K_apply(self._h, float(rho), _dev(psi, (self.V, 4, 3), "psi"),
                                        _dev(out, (self.V, 4, 3), "out"), self._nrhs(psi), prec))
        return out

    def lowmodes_compute(self, rho, n_low, tol=1e-10):
        ev = (ctypes.c_double * n_low)()
        lmax = ctypes.c_double()
        _check(lib().ovl_lowmodes_compute(self._h, float(rho), int(n_low), float(tol), ev,
                                          ctypes.byref(lmax)))
        self.n_low = n_low
        return list(ev), lmax.value

    def kernel_interval(self, rho, max_iter=400):
        """(lmin, lmin_err, lmax): ends of the spectrum of |K| by Lanczos on K^2
        (lmin lies above the true smallest |lambda|; take a margin below it)."""
        lo, err, hi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().ovl_kernel_interval(self._h, float(rho), int(max_iter), ctypes.byref(lo), ctypes.byref(err),
                                         ctypes.byref(hi)))
        return lo.value, err.value, hi.value

    def lowmodes_set(self, evals, evecs):
        n = len(evals)
        ev = (ctypes.c_double * max(n, 1))(*[float(e) for e in evals])
        p = _dev(evecs, (self.V, 4, 3), "evecs") if n else None
        _check(lib().ovl_lowmodes_set(self._h, n, ev, p))
        self.n_low = n

    def lowmodes_get(self):
        out = torch.empty((self.n_low, self.V, 4, 3), dtype=torch.complex128, device="cuda")
        _check(lib().ovl_lowmodes_get(self._h, _dev(out, (self.V, 4, 3), "out")))
        return out

    def sign(self, psi, rho, zolo, eta, prec=F64, allow=()):
        out = torch.empty_like(psi)
        st = Stats()
        code = _check(lib().ovl_sign_zolotarev_mscg(self._h, float(rho), ctypes.byref(zolo),
                                                    _dev(psi, (self.V, 4, 3), "psi"),
                                                    _dev(out, (self.V, 4, 3), "out"),
                                                    self._nrhs(psi), float(eta), prec,
                                                    ctypes.byref(st)), allow)
        return out, st

    def sign_lanczos(self, psi, rho, zolo, eta):
        """sign(K) psi by the two-pass Lanczos method (FP64); zolo gives the interval."""
        out = torch.empty_like(psi)
        st = Stats()
        _check(lib().ovl_sign_lanczos(self._h, float(rho), ctypes.byref(zolo), _dev(psi, (self.V, 4, 3), "psi"),
                                      _dev(out, (self.V, 4, 3), "out"), self._nrhs(psi), float(eta),
                                      ctypes.byref(st)))
        return out, st

    def overlap(self, psi, rho, mu, zolo, eta, prec=F64):
        out = torch.empty_like(psi)
        st = Stats()
        _check(lib().ovl_overlap_apply(self._h, float(rho), float(mu), ctypes.byref(zolo),
                                       _dev(psi, (self.V, 4, 3), "psi"),
                                       _dev(out, (self.V, 4, 3), "out"), self._nrhs(psi),
                                       float(eta), prec, ctypes.byref(st)))
        return out, st

    def overlap_adjoint(self, psi, chi, rho, mu, zolo, eta, prec=F64, want_psi=True, want_links=True):
        """Derivatives of S = sum_f Re(chi_f^H D[mu] psi_f): (D^dagger chi or None,
        link gradient [V,4,3,3] or None, Stats)."""
        nrhs = self._nrhs(chi)
        if want_links and (psi is None or psi.shape != chi.shape):
            raise ValueError("psi and chi must have the same shape")
        dpsi = torch.empty_like(chi) if want_psi else None
        dU = (torch.empty((self.V, 4, 3, 3), dtype=torch.complex128, device=chi.device)
              if want_links else None)
        st = Stats()
        _check(lib().ovl_overlap_adjoint(
            self._h, float(rho), float(mu), ctypes.byref(zolo),
            _dev(psi, (self.V, 4, 3), "psi") if want_links else None,
            _dev(chi, (self.V, 4, 3), "chi"), nrhs, float(eta), prec,
            _dev(dpsi, (self.V, 4, 3), "dpsi") if want_psi else None,
            _dev(dU, (self.V, 4, 3, 3), "dU") if want_links else None, ctypes.byref(st)))
        return dpsi, dU, st

    def solve(self, b, zolo, params, allow=()):
        """GMRESR(relSUMR) solve of D[mu] x = b; returns (x, [Stats per rhs], status)."""
        nrhs = self._nrhs(b)
        x = torch.empty_like(b)
        st = (Stats * nrhs)()
        code = _check(lib().ovl_sumr_gmresr_solve(self._h, ctypes.byref(zolo), ctypes.byref(params),
                                                  _dev(b, (self.V, 4, 3), "b"),
                                                  _dev(x, (self.V, 4, 3), "x"), nrhs, st), allow)
        return x, list(st), code

    # -- eigenspace (eigSUMR, deflation)
    def eigspace_info(self, cap=512):
        n = ctypes.c_int32()
        nd = ctypes.c_int32()
        ritz = (ctypes.c_double * cap)()
        res = (ctypes.c_double * cap)()
        _check(lib().ovl_eigspace_info(self._h, ctypes.byref(n), cap, ritz, res, ctypes.byref(nd)))
        k = min(n.value, cap)
        return {"held": n.value, "ndiag": nd.value, "ritz": list(ritz)[:k], "resid": list(res)[:k]}

    def eigspace_get(self):
        k = self.eigspace_info()["held"]
        v = torch.empty((k, self.V, 4, 3), dtype=torch.complex128, device="cuda")
        vd = torch.empty_like(v)
        if k:
            _check(lib().ovl_eigspace_get(self._h, _dev(v, (self.V, 4, 3), "v"),
                                          _dev(vd, (self.V, 4, 3), "vD")))
        return v, vd

    def eigspace_set(self, n, m, mu, v=None, vD=None, delta=0.1):
        k = 0 if v is None else int(v.shape[0])
        pv = _dev(v, (self.V, 4, 3), "v") if k else None
        pd = _dev(vD, (self.V, 4, 3), "vD") if k else None
        _check(lib().ovl_eigspace_set(self._h, int(n), int(m), float(mu), float(delta), k, pv, pd))

    def eigspace_save(self, path):
        _check(lib().ovl_eigspace_save(self._h, os.fsencode(path)))

    def eigspace_load(self, path):
        _check(lib().ovl_eigspace_load(self._h, os.fsencode(path)))

    def eigspace_diagonalise(self):
        _check(lib().ovl_eigspace_diagonalise(self._h))

    def eigspace_recompute(self, rho, zolo, eta=1e-12):
        _check(lib().ovl_eigspace_recompute(self._h, float(rho), ctypes.byref(zolo), float(eta)))

    def eigensolve(self, q0, zolo, params, max_runs=10, diag_per_run=24, eta_fixed=0.0):
        """Standalone eigSUMR eigensolver from the start vector q0 [V,4,3]; the
        eigenvectors stay in the eigenspace.  Returns (status, per-run list of
        (U applications so far, largest residual), Stats); status -4 when the
        residual target was not reached within max_runs runs."""
        runs = ctypes.c_int32()
        ap = (ctypes.c_int64 * max_runs)()
        mr = (ctypes.c_double * max_runs)()
        st = Stats()
        code = _check(lib().ovl_eigsumr_eigensolve(self._h, ctypes.byref(zolo), ctypes.byref(params),
                                                   _dev(q0, (self.V, 4, 3), "q0"), int(max_runs), int(diag_per_run),
                                                   float(eta_fixed), ctypes.byref(runs), ap, mr,
                                                   ctypes.byref(st)), (-4,))
        return code, [(ap[i], mr[i]) for i in range(runs.value)], st

    def deflate_project(self, b):
        x0 = torch.empty_like(b)
        dx0 = torch.empty_like(b)
        _check(lib().ovl_deflate_project(self._h, _dev(b, (self.V, 4, 3), "b"), _dev(x0, (self.V, 4, 3), "x0"),
                                         _dev(dx0, (self.V, 4, 3), "Dx0"), self._nrhs(b)))
        return x0, dx0

    # -- profiling
    def stream_bench(self, kind, src, dst, reps=20):
        """Average ms per launch of the library's streaming kernel: kind 0 copies
        src into dst (same size), kind 1 reads src (dst: >= 64 KiB scratch)."""
        ms = ctypes.c_double()
        _check(lib().ovl_stream_bench(self._h, int(kind), ctypes.c_void_p(src.data_ptr()),
                                      ctypes.c_void_p(dst.data_ptr()), int(src.numel() * src.element_size()),
                                      int(reps), ctypes.byref(ms)))
        return ms.value

    def set_option(self, option, value):
        _check(lib().ovl_set_option(self._h, int(option), int(bool(value))))

    def gauge_info(self):
        """(largest deviation of the links' third rows from the two-row rebuild,
        whether the FP32 / FP16 stencils use the two-row form)."""
        dev = ctypes.c_double()
        tr = ctypes.c_int32()
        _check(lib().ovl_gauge_info(self._h, ctypes.byref(dev), ctypes.byref(tr)))
        return dev.value, bool(tr.value)

    def tuning(self):
        """The stencil launch variants chosen so far, {key: variant}."""
        n = ctypes.c_int32()
        _check(lib().ovl_tuning_get(self._h, None, None, 0, ctypes.byref(n)))
        k = (ctypes.c_int32 * max(n.value, 1))()
        v = (ctypes.c_int32 * max(n.value, 1))()
        _check(lib().ovl_tuning_get(self._h, k, v, n.value, ctypes.byref(n)))
        return {int(k[i]): int(v[i]) for i in range(n.value)}

    def set_tuning(self, table):
        items = sorted((int(a), int(b)) for a, b in table.items())
        k = (ctypes.c_int32 * max(len(items), 1))(*[a for a, _ in items])
        v = (ctypes.c_int32 * max(len(items), 1))(*[b for _, b in items])
        _check(lib().ovl_tuning_set(self._h, k, v, len(items)))

    def profile(self, on=True):
        _check(lib().ovl_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, kernel, prec):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(lib().ovl_profile_read(self._h, int(kernel), int(prec), ctypes.byref(n),
                                      ctypes.byref(ms), ctypes.byref(by)))
        return {"launches": n.value, "ms": ms.value, "bytes": by.value}


class Instance(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("zolo", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("nrhs", ctypes.c_int32), ("stats", ctypes.c_void_p),
                ("status", ctypes.c_int32), ("message", ctypes.c_char * 160)]


def solve_many(items, params):
    """Solve several instances at once: items = [(ctx, zolo, b), ...] with
    distinct contexts (give each its own stream for the work to overlap).
    Returns [(x, [Stats], status), ...]."""
    n = len(items)
    arr = (Instance * n)()
    keep = []
    for i, (ctx, zolo, b) in enumerate(items):
        nrhs = ctx._nrhs(b)
        x = torch.empty_like(b)
        st = (Stats * nrhs)()
        keep.append((x, st))
        arr[i] = Instance(ctx._h.value if hasattr(ctx._h, "value") else ctx._h, ctypes.addressof(zolo),
                          _dev(b, (ctx.V, 4, 3), "b").value, _dev(x, (ctx.V, 4, 3), "x").value, nrhs,
                          ctypes.addressof(st), 0, b"")
    _check(lib().ovl_sumr_gmresr_solve_many(arr, n, ctypes.byref(params)), allow=(-4,))
    return [(keep[i][0], list(keep[i][1]), arr[i].status) for i in range(n)]


class OverlapFunction(torch.autograd.Function):
    """y = D[mu] psi through the library, differentiable in psi and in the
    links (forward: ovl_overlap_apply; backward: ovl_overlap_adjoint with
    chi = the incoming gradient).  U must be the canonical gauge field that is
    loaded in ctx; it only carries the link gradient.  Usage:
    OverlapFunction.apply(ctx, U, psi, rho, mu, zolo, eta, prec)."""

    @staticmethod
    def forward(fctx, ctx, U, psi, rho, mu, zolo, eta, prec=F64):
        y, _ = ctx.overlap(psi.contiguous(), rho, mu, zolo, eta, prec)
        fctx.save_for_backward(psi)
        fctx.args = (ctx, rho, mu, zolo, eta, F64 if prec == F64 else F32)
        return y

    @staticmethod
    def backward(fctx, gy):
        (psi,) = fctx.saved_tensors
        ctx, rho, mu, zolo, eta, prec = fctx.args
        need_U, need_psi = fctx.needs_input_grad[1], fctx.needs_input_grad[2]
        if not (need_U or need_psi):
            return (None,) * 8
        dpsi, dU, _ = ctx.overlap_adjoint(psi.contiguous(), gy.contiguous(), rho, mu, zolo, eta, prec,
                                          want_psi=need_psi, want_links=need_U)
        return None, dU, dpsi, None, None, None, None, None
