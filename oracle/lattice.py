"""Oracle: the Wilson kernel operator K = gamma_5 D_W(-rho) on the CPU in FP64.

TEST INFRASTRUCTURE ONLY.  Thin ctypes wrapper over ``wilson.c`` (paper
Sec. 1, eq. 2).  Fields are numpy complex128 arrays in canonical layout:
``U[V,4,3,3]``, ``psi[V,4,3]`` (site lexicographic, x fastest).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.ora_gamma.argtypes = [P]
        L.ora_hopping.argtypes = [P, P, P, P]
        L.ora_dw.argtypes = [P, P, ctypes.c_double, P, P]
        L.ora_kernel.argtypes = [P, P, ctypes.c_double, P, P]
        L.ora_kernel_sq_shift.argtypes = [P, P, ctypes.c_double, ctypes.c_double, P, P, P]
        L.ora_hopping_sites.argtypes = [P, P, P, P, ctypes.c_int64, P]
        L.ora_axpy_real.argtypes = [ctypes.c_int64, ctypes.c_double, P, P]
        L.ora_axpby_real.argtypes = [ctypes.c_int64, ctypes.c_double, P, ctypes.c_double, P]
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def _field(a, V):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    assert a.size == V * 12, "spinor size mismatch"
    return a


def volume(dims):
    return int(np.prod(dims))


def gamma():
    """gamma_1..gamma_4 and gamma_5 (chiral basis) as a [5,4,4] array."""
    g = np.zeros((5, 4, 4), np.complex128)
    lib().ora_gamma(_ptr(g))
    return g


G5 = np.array([1.0, 1.0, -1.0, -1.0])


def g5(psi):
    """gamma_5 psi; gamma_5 = diag(1,1,-1,-1) in the chiral basis."""
    psi = np.asarray(psi)
    return psi * G5.reshape((1,) * (psi.ndim - 2) + (4, 1))


class WilsonKernel:
    """K = gamma_5 D_W(-rho) for one gauge field (paper Sec. 1, eq. 2)."""

    def __init__(self, dims, U, rho):
        self.dims = _dims(dims)
        self.V = volume(dims)
        self.U = np.ascontiguousarray(U, dtype=np.complex128).reshape(self.V, 4, 3, 3)
        self.rho = float(rho)
        self.shape = (self.V, 4, 3)
        self.ncalls = 0

    def hop(self, psi):
        psi = _field(psi, self.V).reshape(self.shape)
        out = np.empty_like(psi)
        lib().ora_hopping(_ptr(self.dims), _ptr(self.U), _ptr(psi), _ptr(out))
        self.ncalls += 1
        return out

    def hop_sites(self, psi, sites):
        """(H psi) at the given sites only, shape [len(sites), 4, 3]."""
        psi = _field(psi, self.V).reshape(self.shape)
        sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
        out = np.empty((len(sites), 4, 3), np.complex128)
        lib().ora_hopping_sites(_ptr(self.dims), _ptr(self.U), _ptr(psi), _ptr(sites),
                                len(sites), _ptr(out))
        return out

    def K_sites(self, psi, sites):
        """(K psi) at the given sites: gamma_5 ((4 - rho) psi - H psi / 2)."""
        psi = np.asarray(psi).reshape(self.shape)
        sites = np.asarray(sites, dtype=np.int64)
        return g5((4.0 - self.rho) * psi[sites] - 0.5 * self.hop_sites(psi, sites))

    def dw(self, psi):
        psi = _field(psi, self.V).reshape(self.shape)
        out = np.empty_like(psi)
        lib().ora_dw(_ptr(self.dims), _ptr(self.U), self.rho, _ptr(psi), _ptr(out))
        self.ncalls += 1
        return out

    def K(self, psi):
        psi = _field(psi, self.V).reshape(self.shape)
        out = np.empty_like(psi)
        lib().ora_kernel(_ptr(self.dims), _ptr(self.U), self.rho, _ptr(psi), _ptr(out))
        self.ncalls += 1
        return out

    def K2s(self, psi, sigma=0.0):
        """(K^2 + sigma) psi."""
        psi = _field(psi, self.V).reshape(self.shape)
        tmp = np.empty_like(psi)
        out = np.empty_like(psi)
        lib().ora_kernel_sq_shift(_ptr(self.dims), _ptr(self.U), self.rho, float(sigma),
                                  _ptr(psi), _ptr(tmp), _ptr(out))
        self.ncalls += 2
        return out

    def dense(self, op="K"):
        """Dense matrix of K (or D_W, H) by applying it to unit vectors."""
        n = self.V * 12
        f = {"K": self.K, "dw": self.dw, "hop": self.hop}[op]
        M = np.empty((n, n), np.complex128)
        e = np.zeros(n, np.complex128)
        for j in range(n):
            e[j] = 1.0
            M[:, j] = f(e).reshape(-1)
            e[j] = 0.0
        return M


def dot(a, b):
    """(a, b) = a^dagger b."""
    return np.vdot(a.reshape(-1), b.reshape(-1))


def norm(a):
    return float(np.linalg.norm(a.reshape(-1)))


def _inplace(y, x):
    assert y.dtype == np.complex128 and y.flags.c_contiguous and x.dtype == np.complex128
    assert x.flags.c_contiguous and x.size == y.size


def axpy(a, x, y):
    """y <- y + a x in place (a real), the same values as y + a * x."""
    _inplace(y, x)
    lib().ora_axpy_real(y.size, float(a), _ptr(x), _ptr(y))


def axpby(a, x, b, y):
    """y <- a x + b y in place (a, b real), the same values as a * x + b * y."""
    _inplace(y, x)
    lib().ora_axpby_real(y.size, float(a), _ptr(x), float(b), _ptr(y))
