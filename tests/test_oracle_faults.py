"""Failure handling in the oracle's solvers (CPU): SUMR restarts after loss of
normalisation (Sec. 2, threshold of Sec. 6), the outer iteration limit of
Alg. 3, and deflation from a space whose v^D carries errors (Sec. 4)."""
import numpy as np

import synth
from oracle import eig, krylov
from oracle.lattice import WilsonKernel, g5, norm
from oracle.zolotarev import Zolotarev

MU = 0.05


def _setup(dims=(4, 4, 2, 2), seed=2, eps=0.4):
    k = WilsonKernel(dims, synth.gauge_field(dims, seed, eps), 1.4)
    w, Q = np.linalg.eigh(k.dense("K"))
    z = Zolotarev(16, np.abs(w).min(), np.abs(w).max())
    ov = krylov.Overlap(krylov.SignFunction(k, z), MU)
    n = k.V * 12
    G5 = np.kron(np.eye(k.V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
    D = 0.5 * (1 + MU) * np.eye(n) + 0.5 * (1 - MU) * G5 @ (Q @ np.diag(np.sign(w)) @ Q.conj().T)
    return dims, ov, D, G5


def test_restarts_after_normalisation_loss_still_converge():
    """Relaxed middle solves (U with errors up to 1e-2) and a normalisation
    threshold of 1e-4: SUMR restarts, and GMRESR still reaches 1e-10."""
    dims, ov, D, _ = _setup()
    b = synth.z2_source(dims, 9)
    bn = norm(b)
    rho = (1 - MU) / (1 + MU)
    restarts = []

    def middle(r):
        bp = (2.0 / (1 + MU)) * r
        bpn = norm(bp)
        res = krylov.sumr(ov.U, rho, bp, 1e-3, eta_fn=lambda j, rs: 1e-3 if not rs else min(1e-2, 1e-3 * bpn / rs),
                          norm_restart=1e-4)
        restarts.append(res.restarts)
        return res.x, res.iters

    def apply_A(u):
        return ov(u, min(1e-2, 1e-10 * bn / (2 * (1 - MU) * norm(u))))

    res = krylov.gmresr(apply_A, middle, b, 0.5e-10)
    assert sum(restarts) > 0
    assert norm(b.reshape(-1) - D @ res.x.reshape(-1)) <= 1e-10 * bn


def test_outer_limit_keeps_best_iterate():
    """Alg. 3 stopped after one step returns an iterate that lowers the residual."""
    dims, ov, D, _ = _setup()
    b = synth.z2_source(dims, 10)
    res = krylov.gmresr(lambda u: ov(u, 1e-12),
                        lambda r: (krylov.sumr_overlap(ov, r, 1e-3, maxiter=5).x, 5), b, 1e-10, max_steps=1)
    r = norm(b.reshape(-1) - D @ res.x.reshape(-1)) / norm(b)
    assert res.steps == 1 and np.all(np.isfinite(res.x)) and 1e-10 < r < 1.0


def test_deflation_with_noisy_images_still_converges():
    """Eight exact low eigenvectors of gamma_5 D with v^D errors of relative
    size 1e-2: the deflated GMRESR(relSUMR) solve reaches 1e-10 with the exact D."""
    dims, ov, D, G5 = _setup()
    H = G5 @ D
    h, Y = np.linalg.eigh(0.5 * (H + H.conj().T))
    idx = np.argsort(np.abs(h))[:8]
    rng = np.random.default_rng(3)
    shape = (int(np.prod(dims)), 4, 3)
    vecs, dvecs = [], []
    for j in idx:
        dv = D @ Y[:, j]
        e = rng.normal(size=dv.shape) + 1j * rng.normal(size=dv.shape)
        dvecs.append((dv + 1e-2 * np.linalg.norm(dv) * e / np.linalg.norm(e)).reshape(shape))
        vecs.append(Y[:, j].reshape(shape))
    defl = eig.Deflation(vecs, dvecs)
    b = synth.z2_source(dims, 11)
    res = krylov.gmresr_sumr(ov, b, 1e-10, 1e-3, deflation=defl)
    assert norm(b.reshape(-1) - D @ res.x.reshape(-1)) <= 1e-10 * norm(b)
