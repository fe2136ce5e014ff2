"""Seeded synthetic inputs: gauge fields and sources.

This module is shared input generation only.  It holds none of the overlap
method's arithmetic: it draws SU(3) link variables and source vectors from a
counter-based random number generator, with every floating-point step written
as a fixed sequence of IEEE additions, multiplications, divisions and square
roots, so that a GPU implementation of the same recipe can reproduce it bit for
bit.

Recipe
------
* Random bits: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
  numbers: as easy as 1, 2, 3", SC'11).  Key = the 64-bit seed split in two
  32-bit words; counter = (index, draw, tag, 0).
* Uniform double in [0,1): ``((w0 >> 5) * 2**26 + (w1 >> 6)) * 2**-53``.
* Normal deviates: Box-Muller, ``r = sqrt(-2 ln(1-u1))``, angle ``2 pi u2``,
  with ``ln``, ``sin`` and ``cos`` evaluated by the fixed series below.
* Link variable: ``U = exp(i eps A)``, ``A = sum_a g_a T^a``, ``T^a`` the
  Gell-Mann matrices over two, ``g_a ~ N(0,1)`` (8 deviates per link).  The
  exponential is a degree-14 Taylor polynomial of ``X/16`` in Horner form,
  squared four times.
* Layouts are the canonical ones: ``U[site][mu][a][b]`` and
  ``psi[site][spin][colour]``, complex128, site lexicographic with x fastest.
"""
import concurrent.futures
import os

import numpy as np

M32 = np.uint64(0xFFFFFFFF)
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)

TAG_GAUGE = 0x47415547  # "GAUG"
TAG_GAUSS = 0x53524347  # "GCRS"
TAG_Z2 = 0x5A32534E     # "NS2Z"

LN2 = 0.6931471805599453
PI_4 = 0.7853981633974483


def philox4x32(c0, c1, c2, c3, seed):
    """Philox4x32-10 on uint64 arrays holding 32-bit words; returns 4 words."""
    c0 = np.asarray(c0, np.uint64) & M32
    c1 = np.asarray(c1, np.uint64) & M32
    c2 = np.asarray(c2, np.uint64) & M32
    c3 = np.asarray(c3, np.uint64) & M32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    k0 = np.uint64(int(seed) & 0xFFFFFFFF)
    k1 = np.uint64((int(seed) >> 32) & 0xFFFFFFFF)
    for rnd in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & M32
        hi1, lo1 = p1 >> np.uint64(32), p1 & M32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & M32, lo1, (hi0 ^ c3 ^ k1) & M32, lo0
        if rnd < 9:
            k0 = (k0 + PHILOX_W0) & M32
            k1 = (k1 + PHILOX_W1) & M32
    return c0, c1, c2, c3


def uniform53(w0, w1):
    """Two 32-bit words -> double in [0,1) with 53 random bits (exact)."""
    a = (w0 >> np.uint64(5)).astype(np.float64)
    b = (w1 >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b) * (1.0 / 9007199254740992.0)


def _log_unit(u):
    """ln(u) for u in (0,1]: u = m 2^e, m in [sqrt(1/2), sqrt(2)),
    ln m = 2 atanh(z), z = (m-1)/(m+1), atanh by its odd power series."""
    m, e = np.frexp(u)
    small = m < 0.7071067811865476
    m = np.where(small, m * 2.0, m)
    e = np.where(small, e - 1, e).astype(np.float64)
    z = (m - 1.0) / (m + 1.0)
    z2 = z * z
    s = np.full_like(z, 1.0 / 25.0)
    for k in range(11, -1, -1):
        s = (1.0 / (2 * k + 1)) + z2 * s
    return e * LN2 + (2.0 * z) * s


def _sin_poly(t):
    t2 = t * t
    s = np.full_like(t, 1.0)
    for k in range(10, 0, -1):
        s = 1.0 - (t2 * (1.0 / ((2 * k) * (2 * k + 1)))) * s
    return t * s


def _cos_poly(t):
    t2 = t * t
    s = np.full_like(t, 1.0)
    for k in range(10, 0, -1):
        s = 1.0 - (t2 * (1.0 / ((2 * k - 1) * (2 * k)))) * s
    return s


def _sincos_2pi(u):
    """(sin 2 pi u, cos 2 pi u) for u in [0,1) by octant reduction."""
    v = u * 8.0
    k = np.floor(v)
    f = v - k
    k = k.astype(np.int64)
    odd = (k & 1) == 1
    t = np.where(odd, 1.0 - f, f) * PI_4
    st, ct = _sin_poly(t), _cos_poly(t)
    sa = np.where(odd, ct, st)
    ca = np.where(odd, st, ct)
    q = k >> 1
    s = np.select([q == 0, q == 1, q == 2], [sa, ca, -sa], -ca)
    c = np.select([q == 0, q == 1, q == 2], [ca, -sa, -ca], sa)
    return s, c


def box_muller(u1, u2):
    """Two uniforms in [0,1) -> two N(0,1) deviates."""
    r = np.sqrt(-2.0 * _log_unit(1.0 - u1))
    s, c = _sincos_2pi(u2)
    return r * c, r * s


def normals(index, draws, tag, seed):
    """2*draws normal deviates per index, shape (len(index), 2*draws).  Draw d
    is one Philox call with counter (index, d, tag, 0); its four words give the
    two uniforms of one Box-Muller pair, stored as columns 2d and 2d+1."""
    index = np.asarray(index, np.uint64)
    out = []
    for d in range(draws):
        w0, w1, w2, w3 = philox4x32(index, np.uint64(d), np.uint64(tag), np.uint64(0), seed)
        ua, ub = uniform53(w0, w1), uniform53(w2, w3)
        za, zb = box_muller(ua, ub)
        out += [za, zb]
    return np.stack(out, axis=-1)


# Gell-Mann matrices lambda_a; T^a = lambda_a / 2.
def gell_mann():
    lam = np.zeros((8, 3, 3), complex)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3.0)
    lam[7][2, 2] = -2 / np.sqrt(3.0)
    return lam


INV_SQRT3 = 0.5773502691896258  # 1/sqrt(3) as a double literal


def _su3_algebra(g, eps):
    """X = i eps sum_a g_a lambda_a / 2 as (re, im) arrays [..., 3, 3], each
    entry built by a fixed sequence of real operations."""
    h = 0.5 * eps
    a = [g[..., i] * h for i in range(8)]   # eps/2 g_a
    re = np.zeros(g.shape[:-1] + (3, 3))
    im = np.zeros(g.shape[:-1] + (3, 3))
    # A = sum a_i lambda_i (Hermitian);  X = i A: re(X) = -im(A), im(X) = re(A)
    # A entries:
    A_re = np.zeros_like(re)
    A_im = np.zeros_like(re)
    A_re[..., 0, 0] = a[2] + a[7] * INV_SQRT3
    A_re[..., 1, 1] = (0.0 - a[2]) + a[7] * INV_SQRT3
    A_re[..., 2, 2] = a[7] * (-2.0 * INV_SQRT3)
    A_re[..., 0, 1] = a[0]
    A_im[..., 0, 1] = 0.0 - a[1]
    A_re[..., 1, 0] = a[0]
    A_im[..., 1, 0] = a[1]
    A_re[..., 0, 2] = a[3]
    A_im[..., 0, 2] = 0.0 - a[4]
    A_re[..., 2, 0] = a[3]
    A_im[..., 2, 0] = a[4]
    A_re[..., 1, 2] = a[5]
    A_im[..., 1, 2] = 0.0 - a[6]
    A_re[..., 2, 1] = a[5]
    A_im[..., 2, 1] = a[6]
    re = 0.0 - A_im
    im = A_re.copy()
    return re, im


def _cmatmul3(ar, ai, br, bi):
    """3x3 complex product with a fixed summation order (k = 0, 1, 2)."""
    cr = np.empty_like(ar)
    ci = np.empty_like(ai)
    for i in range(3):
        for j in range(3):
            sr = ar[..., i, 0] * br[..., 0, j] - ai[..., i, 0] * bi[..., 0, j]
            si = ar[..., i, 0] * bi[..., 0, j] + ai[..., i, 0] * br[..., 0, j]
            for k in (1, 2):
                sr = sr + (ar[..., i, k] * br[..., k, j] - ai[..., i, k] * bi[..., k, j])
                si = si + (ar[..., i, k] * bi[..., k, j] + ai[..., i, k] * br[..., k, j])
            cr[..., i, j] = sr
            ci[..., i, j] = si
    return cr, ci


EXP_SQUARINGS = 4
EXP_DEGREE = 14


def su3_exp(xr, xi):
    """exp(X) for anti-Hermitian X by scaling, Taylor (Horner) and squaring."""
    sc = 1.0 / (1 << EXP_SQUARINGS)
    xr = xr * sc
    xi = xi * sc
    eye = np.broadcast_to(np.eye(3), xr.shape)
    pr = eye.copy()
    pi = np.zeros_like(xi)
    for k in range(EXP_DEGREE, 0, -1):
        tr, ti = _cmatmul3(xr, xi, pr, pi)
        inv = 1.0 / k
        pr = eye + tr * inv
        pi = ti * inv
    for _ in range(EXP_SQUARINGS):
        pr, pi = _cmatmul3(pr, pi, pr, pi)
    return pr, pi


def volume(dims):
    d = [int(v) for v in dims]
    return d[0] * d[1] * d[2] * d[3]


def gauge_field(dims, seed, eps, chunk=1 << 16, workers=None):
    """U_mu(x) = exp(i eps sum_a g_a T^a), canonical complex128 [V,4,3,3].

    Links are independent (each has its own counter), so chunks of links are
    generated by a pool of threads; every link goes through the same sequence
    of operations whatever the chunking, so the field is the same bit for bit."""
    V = volume(dims)
    nlink = 4 * V
    out = np.empty((nlink, 3, 3), np.complex128)

    def work(s):
        idx = np.arange(s, min(nlink, s + chunk), dtype=np.uint64)
        g = normals(idx, 4, TAG_GAUGE, seed)   # 8 deviates per link
        xr, xi = _su3_algebra(g, eps)
        ur, ui = su3_exp(xr, xi)
        out[s:s + len(idx)] = ur + 1j * ui

    starts = range(0, nlink, chunk)
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or nlink <= chunk:
        for s in starts:
            work(s)
    else:
        with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(work, starts))
    return out.reshape(V, 4, 3, 3)


def gauge_links(link_index, seed, eps):
    """The links with flat indices site*4 + mu only, [n,3,3] (same values as gauge_field)."""
    idx = np.asarray(link_index, dtype=np.uint64)
    g = normals(idx, 4, TAG_GAUGE, seed)
    xr, xi = _su3_algebra(g, eps)
    ur, ui = su3_exp(xr, xi)
    return ur + 1j * ui


def unit_gauge(dims):
    V = volume(dims)
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()


def point_source(dims, site=0, spin=0, colour=0):
    V = volume(dims)
    b = np.zeros((V, 4, 3), np.complex128)
    b[site, spin, colour] = 1.0
    return b


def gaussian_source(dims, seed):
    """Each complex component: Re, Im independent N(0,1)."""
    V = volume(dims)
    n = V * 12
    idx = np.arange(n, dtype=np.uint64)
    g = normals(idx, 1, TAG_GAUSS, seed)
    return (g[:, 0] + 1j * g[:, 1]).reshape(V, 4, 3)


def z2_source(dims, seed):
    """Each real component +-1 with equal probability."""
    V = volume(dims)
    n = V * 12
    idx = np.arange(n, dtype=np.uint64)
    w0, w1, _, _ = philox4x32(idx, np.uint64(0), np.uint64(TAG_Z2), np.uint64(0), seed)
    re = 1.0 - 2.0 * (w0 & np.uint64(1)).astype(np.float64)
    im = 1.0 - 2.0 * (w1 & np.uint64(1)).astype(np.float64)
    return (re + 1j * im).reshape(V, 4, 3)


def instance_eps(n, seed, lo=0.2, hi=0.35):
    """n link-width parameters uniform in [lo, hi) (batched uneven workload)."""
    w0, w1, _, _ = philox4x32(np.arange(n, dtype=np.uint64), np.uint64(0),
                              np.uint64(0x45505331), np.uint64(0), seed)
    return lo + (hi - lo) * uniform53(w0, w1)
