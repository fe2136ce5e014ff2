"""Benchmark: overlap solves per second at a 1e-10 residual on one MI355X.

Headline workload (one "step" = one complete mixed-precision, eigSUMR-deflated
GMRESR(relSUMR) solve of D[mu] x = b for one spin-colour point source):
24^3 x 48 lattice, links exp(i 0.25 A) (seed 3), K = gamma_5 D_W(-1.4),
mu = 0.01, order-20 Zolotarev sign function on the Lanczos interval of |K|
(no kernel modes need exact treatment there: the spectrum of |K| starts at
0.62), eigSUMR deflation with 20 eigenvectors (Secs. 4-5), target
||b - D x|| <= 1e-10 ||b||.  The steps cycle through the twelve spin-colour
point sources at the origin.  Set-up (gauge field, interval, Zolotarev
coefficients, the eigSUMR calculating solves that build the eigenspace and
its FP64 recomputation) is outside the timed region and reported separately,
with the rate including it and the number of sources at which it pays.
Precision ladder: FP16-storage sign function while the accuracy asked for is
>= 3e-3, FP32 while >= 1e-6, FP64 below; FP64 outer GMRESR, Gram/Rayleigh-Ritz
and projection.  Beside it (not timed steps): the same sources solved
undeflated and with an all-FP64 sign function (medians of three), the
deflation gain in SUMR iterations and time, the eigenvalue ratio of the
deflated space, the 16^3 x 32 plain method (mixed and FP64), the stencil alone
beyond the Infinity Cache, the library's streaming kernels, and the CPU oracle
on a bounded sample of the headline workload.

The timed steps run with profiling off.  Kernel times come from HIP events
attached to each launch's dispatch packet (see ovl_profile_enable), collected
over one replica of a timed solve run right after them.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "overlap solves/s at 1e-10 resid (mixed vs FP64) + Dslash HBM GB/s % peak"
HBM_PEAK_GBS = 8000.0
VALU_ISSUE_PEAK = 256 * 2.4   # G wave instructions/s: 256 CUs, one vector wave instruction per clock each
DIMS = (16, 16, 16, 32)
RHO, MU, NZ, NLOW, TOL = 1.4, 0.02, 20, 10, 1e-10
# middle-solve accuracy of GMRESR for the 16^3 x 32 workload, tuned as Alg. 3
# asks (a sweep over 3e-4 .. 1e-2 on this workload: 3e-3 fastest)
ETA_TILDE_C2 = 3e-3
PREC_NAMES = ("f64", "f32", "f16")
KERN_NAMES = ("stencil", "shift_update")
# sources whose kernels the hardware-counter traffic figures describe
KERNEL_SOURCES = ["dslash.hip", "mscg.hip", "fields.h", "kernels.h", "mscg_state.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison solves on 24^3x48")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 24^3x48 headline and its comparison solves, plus the legs other flags ask for "
                         "(no CPU baseline)")
    ap.add_argument("--extras", action="store_true",
                    help="add the 24 uneven instances, the 4^4 plain method and the adjoint legs")
    ap.add_argument("--batch12", action="store_true",
                    help="add the twelve 24^3x48 point sources deflated in one batched call")
    ap.add_argument("--half-threshold", type=float, default=3e-3,
                    help="16^3x32 leg: sign accuracies at or above this use FP16 storage (> 1 disables)")
    ap.add_argument("--c3-eta", type=float, default=3e-3, help="24^3x48: middle-solve accuracy eta~ of GMRESR")
    ap.add_argument("--relax-cap", type=float, default=3e-2,
                    help="24^3x48: loosest sign accuracy of the relaxed middle solves (Sec. 3: tuned per ensemble)")
    ap.add_argument("--eig-calc", type=int, default=3, help="24^3x48: eigSUMR calculating solves")
    ap.add_argument("--eig-n", type=int, default=20, help="24^3x48: eigenvectors kept (n)")
    ap.add_argument("--eig-m", type=int, default=200, help="24^3x48: basis size of Alg. 6 (m)")
    ap.add_argument("--eig-eps", type=float, default=1e-4, help="24^3x48: target eigenvector accuracy (Sec. 6)")
    ap.add_argument("--eig-block", action="store_true",
                    help="24^3x48: the calculating solves as one batched call collecting into one basis "
                         "(block eigSUMR) instead of one after another")
    ap.add_argument("--full-links", action="store_true",
                    help="24^3x48: FP32 / FP16 stencils on the full 18-real links instead of two rows")
    ap.add_argument("--fixed-nz", action="store_true",
                    help="24^3x48: every sign call with all 20 poles (default: the Zolotarev order per sign call "
                         "from its accuracy, Sec. 3)")
    ap.add_argument("--outer-printed", action="store_true",
                    help="24^3x48: GMRESR outer products c = D u to the accuracy Alg. 3 prints, "
                         "||D u - c|| < eps ||b|| ||u|| / ||r|| (default: eps ||b|| / 4)")
    ap.add_argument("--bound-text", action="store_true",
                    help="24^3x48: eq. (bound) with chi scaling the whole bound (default: as printed, chi on the "
                         "square root only)")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for hardware counters: a 1 GiB elementwise copy (calibration), one "
                         "sign-function call per precision on the 24^3x48 workload, the stand-alone 32^3x64 "
                         "stencil and the 12-field 24^3x48 stencil")
    ap.add_argument("--variant-sweep", action="store_true",
                    help="only: time every stencil launch variant on the 12-field 24^3x48 and 1-field 32^3x64 "
                         "stencils (also the hardware-counter run for them)")
    ap.add_argument("--sign-methods", action="store_true",
                    help="add the comparison of the multi-shift CG and two-pass Lanczos sign functions")
    ap.add_argument("--eigcg", action="store_true",
                    help="add the GMRESR(eigCG) leg on 16^3x32 (calculating solves, then deflated solves)")
    ap.add_argument("--eigcg-calc", type=int, default=5, help="eigCG leg: calculating solves")
    ap.add_argument("--eigsolve", action="store_true",
                    help="add the standalone eigSUMR eigensolver leg on 16^3x32 (relaxed and full accuracy)")
    ap.add_argument("--tuning", default=None,
                    help="JSON of stencil launch choices to install instead of autotuning (the 'tuning' "
                         "object an earlier run printed), so that profiler runs see the same kernels")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_1501_01855_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def setup_c2(ovl, tuning=None):
    ctx = ovl.Context(DIMS)
    if tuning:   # launch choices of an earlier run, installed before any launch
        ctx.set_tuning(tuning["16x16x16x32"])
    ctx.gauge_generate(2, 0.25)
    ev, lmax = ctx.lowmodes_compute(RHO, NLOW, tol=1e-10)
    zolo = ovl.zolotarev_coeffs(NZ, max(abs(e) for e in ev), lmax)
    b = ctx.source(ovl.SRC_GAUSS, seed=102)
    return ctx, zolo, b


def profile_run(torch, ovl, tuning, args):
    """Hardware-counter run (rocprofv3 --pmc): every kernel here is a kernel
    the benchmark times, launched in the same configuration (tuning: the
    benchmark's launch choices, installed before any launch)."""
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    src.fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)   # reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    del src, dst
    ctx, zolo, B, _ = c3_setup(torch, ovl, tuning)
    out = {"calibration_bytes_each_way": 1 << 30}
    for prec in (ovl.HALF, ovl.F32, ovl.F64):
        _, st = ctx.sign(B[0], RHO, zolo, 1e-2, prec=prec)
        out[f"mscg_iters_{PREC_NAMES[prec]}"] = st.mscg_iters
    torch.cuda.synchronize()
    Bs = torch.stack(B)
    for prec in (ovl.F32, ovl.HALF):   # the 12-field stencil of the batched form
        for _ in range(10):
            ctx.wilson_dslash(Bs, prec)
    torch.cuda.synchronize()
    ctx.close()
    ctx = ovl.Context((32, 32, 32, 64))
    ctx.gauge_generate(5, 0.25)
    if tuning and "32x32x32x64" in tuning:
        ctx.set_tuning(tuning["32x32x32x64"])
    psi = ctx.source(ovl.SRC_GAUSS, seed=7)
    for prec in (ovl.F32, ovl.HALF):
        for _ in range(10):
            ctx.wilson_dslash(psi, prec)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps(out), flush=True)


def solve_params(ovl, mixed, half_threshold=2.0):
    return ovl.solver_defaults(rho=RHO, mu=MU, tol=TOL, eta_tilde=ETA_TILDE_C2, relax_floor=1e-2,
                               f32_threshold=(1e-6 if mixed else 10.0),
                               half_threshold=(half_threshold if mixed else 10.0), max_outer=16,
                               max_middle=4000, max_mscg=20000)


def read_prof(ctx, ovl):
    return {(k, p): ctx.profile_read(k, p) for k in (ovl.KERN_STENCIL, ovl.KERN_SHIFT) for p in range(3)}


def time_solves(torch, ctx, ovl, b, zolo, params, steps, warmup):
    """Wall time of `steps` solves with profiling off (the production path),
    then one more solve of the same input with per-launch events on: the
    kernels, their launch shapes and the iteration counts are those of the
    timed solves (the events themselves add about a third to the wall time,
    so they stay out of the timed steps)."""
    for _ in range(warmup):
        ctx.solve(b, zolo, params)
    torch.cuda.synchronize()
    ctx.profile(False)
    t0 = time.perf_counter()
    stats = []
    x = None
    for _ in range(steps):
        x, st, _ = ctx.solve(b, zolo, params)
        stats.append(st[0].as_dict())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.profile(True)
    t1 = time.perf_counter()
    _, stp, _ = ctx.solve(b, zolo, params)
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - t1
    prof = read_prof(ctx, ovl)
    ctx.profile(False)
    if stp[0].mscg_iters != stats[-1]["mscg_iters"]:
        print("[bench] warning: the profiled replica took a different number of iterations",
              file=sys.stderr, flush=True)
    return dt, stats, prof, x, dt_prof


def kernel_summary(prof):
    out = {}
    for (k, p), s in prof.items():
        if not s["launches"]:
            continue
        out[f"{KERN_NAMES[k]}_{PREC_NAMES[p]}"] = {
            "launches": s["launches"], "ms": s["ms"], "avg_us": 1e3 * s["ms"] / s["launches"],
            "bytes_per_launch": s["bytes"] / s["launches"],
            "GBps": s["bytes"] / (s["ms"] * 1e6) if s["ms"] else None}
    return out


def read_counter(kind, name, path):
    """A per-launch figure of kernel slot `name` from the committed
    hardware-counter summary (kind "traffic": HBM-side bytes; "valu": vector
    wave instructions), if it was taken on the current kernel sources."""
    try:
        with open(path) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None, "no counter summary"
    want = kernel_source_hash()
    src = [ln.split()[-1] for ln in lines if ln.startswith("kernel_sources_sha256")]
    if not src or src[0] != want:
        return None, "kernel sources changed since the counters were taken"
    for ln in lines:
        f = ln.split()
        if len(f) >= 3 and f[0] == kind and f[1] == name:
            return float(f[2]), ("rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, calibrated" if kind == "traffic"
                                 else "rocprofv3 --pmc SQ_INSTS_VALU")
    return None, "slot not in the counter summary"


def read_traffic(name, path):
    return read_counter("traffic", name, path)


def uneven_leg(torch, ovl):
    """Twenty-four independent instances, six each of 8^4, 8^3x16, 12^3x24 and
    16^4 (links exp(i eps A), eps uniform in [0.2, 0.35] from seed 4, gauge seed
    400 + i), Z2 sources (seed 104 + i), mu = 0.03, N_Z = 20 with 10 exact kernel
    modes, mixed precision, 1e-10: solved together (one context and stream
    each) and, for comparison, one after another."""
    import synth
    eps = synth.instance_eps(24, 4)
    sizes = [(8, 8, 8, 8), (8, 8, 8, 16), (12, 12, 12, 24), (16, 16, 16, 16)]
    t0 = time.perf_counter()
    items = []
    for i in range(24):
        dims = sizes[i // 6]
        ctx = ovl.Context(dims, stream=torch.cuda.Stream())
        ctx.gauge_generate(400 + i, float(eps[i]))
        ev, lmax = ctx.lowmodes_compute(RHO, NLOW, tol=1e-10)
        zolo = ovl.zolotarev_coeffs(NZ, max(abs(e) for e in ev), lmax)
        items.append((ctx, zolo, ctx.source(ovl.SRC_Z2, seed=104 + i)))
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    p = ovl.solver_defaults(rho=RHO, mu=0.03, tol=TOL, eta_tilde=1e-3, relax_floor=1e-2, f32_threshold=1e-6,
                            half_threshold=3e-3, max_outer=16, max_middle=4000, max_mscg=20000)
    ovl.solve_many(items, p)   # warm-up (autotuning, workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ovl.solve_many(items, p)
    torch.cuda.synchronize()
    together = time.perf_counter() - t0
    t0 = time.perf_counter()
    for ctx, zolo, b in items:
        ctx.solve(b, zolo, p)
    torch.cuda.synchronize()
    alone = time.perf_counter() - t0
    worst = 0.0
    for (ctx, zolo, b), (x, st, code) in zip(items, res):
        Dx, _ = ctx.overlap(x, RHO, 0.03, zolo, 1e-13)
        worst = max(worst, float(torch.linalg.vector_norm(b - Dx) / torch.linalg.vector_norm(b)))
    for ctx, _, _ in items:
        ctx.close()
    return {"instances": "6 each of 8^4, 8^3x16, 12^3x24, 16^4", "setup_s": setup,
            "together_s": together, "solves_per_s_together": 24 / together,
            "one_after_another_s": alone, "solves_per_s_one_after_another": 24 / alone,
            "speedup": alone / together, "max_true_relres": worst,
            "status": [r[2] for r in res]}


def eigcg_leg(torch, ovl, n_calc=5, n_eig=20, m_eig=60):
    """GMRESR(eigCG) on the 16^3 x 32 workload (Sec. 5 collection on the relCG
    middle solve, the Sec. 4 spectral preconditioner from the vectors held):
    n_calc calculating solves on spin-colour point sources at site 0, then a
    fresh point source solved four ways -- relCG preconditioned with the
    eigCG vectors, relCG undeflated, relSUMR started from the same vectors'
    deflation projection, relSUMR undeflated -- all mixed precision to 1e-10."""
    ctx, zolo, _ = setup_c2(ovl)
    B = torch.stack([ctx.source(ovl.SRC_POINT, site=0, spin=i % 4, colour=i % 3) for i in range(n_calc + 1)])

    def params(cg, calc, defl):
        p = solve_params(ovl, True, 3e-3)
        p.middle_cg, p.eig_calc, p.use_deflation = cg, calc, defl
        p.n_eig, p.m_eig, p.eta_tilde, p.verbose = n_eig, m_eig, 1e-3, 1
        return p

    def run(b, p):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, code = ctx.solve(b, zolo, p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        Dx, _ = ctx.overlap(x, RHO, MU, zolo, 1e-13)
        res = float(torch.linalg.vector_norm(b - Dx) / torch.linalg.vector_norm(b))
        d = st[0].as_dict()
        return {"status": code, "seconds": dt, "true_relres": res, "cg_or_sumr_iters": d["sumr_iters"],
                "sign_calls": d["sign_calls"], "mscg_iters": d["mscg_iters"], "gmresr_steps": d["gmresr_steps"]}

    out = {"lattice": "16x16x16x32", "mu": MU, "n_eig": n_eig, "m_eig": m_eig, "calculating": []}
    for i in range(n_calc):
        out["calculating"].append(run(B[i:i + 1], params(1, 1, 1)))
        print(f"[bench] eigCG calculating solve {i} done", file=sys.stderr, flush=True)
    info = ctx.eigspace_info()
    out["eigenspace"] = {"held": info["held"], "diagonalisations": info["ndiag"],
                         "ritz": info["ritz"], "resid": info["resid"]}
    b = B[n_calc:n_calc + 1]
    out["relcg_preconditioned"] = run(b, params(1, 0, 1))
    out["relcg_undeflated"] = run(b, params(1, 0, 0))
    out["relsumr_deflated_start"] = run(b, params(0, 0, 1))
    out["relsumr_undeflated"] = run(b, params(0, 0, 0))
    print("[bench] eigCG comparison solves done", file=sys.stderr, flush=True)
    ctx.close()
    return out


def eigsolve_leg(torch, ovl, n_eig=30, m_eig=110, runs=8):
    """The standalone eigSUMR eigensolver on the 16^3 x 32 workload (Sec. 6's
    set-up: 30 eigenvectors and 80 further basis vectors, restart after 24
    diagonalisations, target residual 1e-4), from a Z2 start, once with the
    Sec. 5.1 relaxation (mixed-precision sign calls) and once at sign accuracy
    1e-10 (FP64): U applications, seconds and the largest residual after
    each run; then the benchmark's Gaussian source solved with the
    eigenvectors found (relSUMR from the deflated start, relCG with the
    spectral preconditioner) and, once, without them."""
    out = {"lattice": "16x16x16x32", "mu": MU, "n_eig": n_eig, "m_eig": m_eig}

    def solve_with(ctx, zolo, b, cg, defl):
        p = solve_params(ovl, True, 3e-3)
        p.middle_cg, p.use_deflation, p.n_eig, p.m_eig = cg, defl, n_eig, m_eig
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, code = ctx.solve(b, zolo, p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        Dx, _ = ctx.overlap(x, RHO, MU, zolo, 1e-13)
        return {"status": code, "seconds": dt, "middle_iters": st[0].sumr_iters,
                "true_relres": float(torch.linalg.vector_norm(b - Dx) / torch.linalg.vector_norm(b))}

    for name, eta in (("relaxed", 0.0), ("full_accuracy", 1e-10)):
        ctx, zolo, b = setup_c2(ovl)
        q0 = ctx.source(ovl.SRC_Z2, seed=103)
        p = solve_params(ovl, eta == 0.0, 3e-3)
        p.n_eig, p.m_eig, p.eig_eps, p.verbose = n_eig, m_eig, 1e-4, 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code, hist, st = ctx.eigensolve(q0, zolo, p, max_runs=runs, diag_per_run=24, eta_fixed=eta)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        info = ctx.eigspace_info()
        d = st.as_dict()
        out[name] = {"status": code, "seconds": dt, "runs": [{"u_applications": a, "max_residual": m} for a, m in hist],
                     "sign_calls": d["sign_calls"], "mscg_iters": d["mscg_iters"],
                     "ritz": sorted(info["ritz"]), "residuals": info["resid"],
                     "relsumr_deflated_start": solve_with(ctx, zolo, b, 0, 1),
                     "relcg_preconditioned": solve_with(ctx, zolo, b, 1, 1)}
        if name == "relaxed":
            out["relsumr_undeflated"] = solve_with(ctx, zolo, b, 0, 0)
            out["relcg_undeflated"] = solve_with(ctx, zolo, b, 1, 0)
        print(f"[bench] eigensolver ({name}) done in {dt:.1f} s", file=sys.stderr, flush=True)
        ctx.close()
    return out


def c1_leg(torch, ovl, reps=10):
    """The plain method on 4^4 (links eps 0.3 seed 1, rho 1.4, N_Z = 16 on
    [lambda_min, lambda_max] of |K| from the GPU's Lanczos, no exact modes,
    mu = 0.05, point source at site 0 spin 0 colour 0, GMRESR(relSUMR) to
    1e-10): solves/s in FP64 and with the precision ladder."""
    ctx = ovl.Context((4, 4, 4, 4))
    ctx.gauge_generate(1, 0.3)
    ev, lmax = ctx.lowmodes_compute(RHO, 1, tol=1e-12)
    ctx.lowmodes_set([], None)   # the interval only; no exactly treated mode
    zolo = ovl.zolotarev_coeffs(16, abs(ev[0]), lmax)
    b = ctx.source(ovl.SRC_POINT, site=0, spin=0, colour=0)
    out = {"lattice": "4^4", "interval": [abs(ev[0]), lmax]}
    for name, mixed in (("fp64", False), ("mixed", True)):
        p = ovl.solver_defaults(rho=RHO, mu=0.05, tol=TOL, eta_tilde=1e-3, f32_threshold=(1e-6 if mixed else 10.0))
        ctx.solve(b, zolo, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            x, st, code = ctx.solve(b, zolo, p)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        Dx, _ = ctx.overlap(x, RHO, 0.05, zolo, 1e-14)
        out[name] = {"status": code, "seconds": dt, "solves_per_s": 1.0 / dt,
                     "true_relres": float(torch.linalg.vector_norm(b - Dx) / torch.linalg.vector_norm(b)),
                     "sumr_iters": st[0].sumr_iters, "mscg_iters": st[0].mscg_iters}
    ctx.close()
    return out


def adjoint_leg(torch, ovl):
    """dS/dpsi and dS/dU for S = Re(chi^H D psi), N_Z = 20, no exactly treated
    modes: 8^3 x 16 in FP64 (eta 1e-10) and 32^3 x 64 in FP32 (eta 1e-6)."""
    out = {}
    ctx = ovl.Context((8, 8, 8, 16))
    ctx.gauge_generate(5, 0.25)
    ev, lmax = ctx.lowmodes_compute(RHO, 1, tol=1e-10)
    ctx.lowmodes_set([], None)
    a = abs(ev[0])
    zolo = ovl.zolotarev_coeffs(NZ, a, lmax)
    for dims, prec, eta, reps in (((8, 8, 8, 16), ovl.F64, 1e-10, 3), ((32, 32, 32, 64), ovl.F32, 1e-6, 1)):
        if dims != (8, 8, 8, 16):
            ctx.close()
            ctx = ovl.Context(dims)
            ctx.gauge_generate(5, 0.25)
        psi = ctx.source(ovl.SRC_GAUSS, seed=105)
        chi = ctx.source(ovl.SRC_GAUSS, seed=106)
        ctx.overlap_adjoint(psi, chi, RHO, 0.05, zolo, eta, prec)   # warm-up (autotuning)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, _, st = ctx.overlap_adjoint(psi, chi, RHO, 0.05, zolo, eta, prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out["x".join(map(str, dims))] = {"prec": PREC_NAMES[prec], "eta": eta, "seconds": dt,
                                        "adjoints_per_s": 1.0 / dt, "mscg_iters": st.mscg_iters}
    out["interval"] = [a, lmax]
    ctx.close()
    return out


def _stencil_rates(torch, ovl, ctx, psi, reps):
    res = {}
    for prec in (ovl.F32, ovl.HALF):
        ctx.wilson_dslash(psi, prec)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            ctx.wilson_dslash(psi, prec)
        torch.cuda.synchronize()
        p = ctx.profile_read(ovl.KERN_STENCIL, prec)
        ctx.profile(False)
        gbs = p["bytes"] / (p["ms"] * 1e6)
        res[PREC_NAMES[prec]] = {"launches": p["launches"], "avg_us": 1e3 * p["ms"] / p["launches"],
                                 "bytes_per_launch": p["bytes"] / p["launches"], "GBps": gbs,
                                 "frac_of_peak": gbs / HBM_PEAK_GBS}
    return res


def dslash_alone(torch, ovl, tuning=None, reps=50):
    """The hopping stencil alone (FP32 and FP16 storage) on 32^3 x 64 (links
    seed 5, one Gaussian field) and, in its batched form, on twelve fields of
    24^3 x 48 (links seed 3): algorithmic bytes are the spinors in and out of
    every field plus one read of the links per launch."""
    ctx = ovl.Context((32, 32, 32, 64))
    if tuning and "32x32x32x64" in tuning:
        ctx.set_tuning(tuning["32x32x32x64"])
    ctx.gauge_generate(5, 0.25)
    psi = ctx.source(ovl.SRC_GAUSS, seed=7)
    res = {"lattice": "32^3x64", "two_row_links": ctx.gauge_info()[1], **_stencil_rates(torch, ovl, ctx, psi, reps)}
    res["tuning"] = {"32x32x32x64": ctx.tuning()}
    ctx.close()
    # the same with the full 18-real links (fresh context: its own launch choices)
    ctx = ovl.Context((32, 32, 32, 64))
    ctx.set_option(ovl.OPT_TWO_ROW_LINKS, 0)
    ctx.gauge_generate(5, 0.25)
    psi = ctx.source(ovl.SRC_GAUSS, seed=7)
    res["full_links"] = _stencil_rates(torch, ovl, ctx, psi, reps)
    res["full_links"]["tuning"] = ctx.tuning()
    ctx.close()
    ctx = ovl.Context((24, 24, 24, 48))
    if tuning and "24x24x24x48" in tuning:
        ctx.set_tuning(tuning["24x24x24x48"])
    ctx.gauge_generate(3, 0.25)
    B = torch.stack([ctx.source(ovl.SRC_GAUSS, seed=300 + f) for f in range(12)])
    res["fields12_24c48"] = _stencil_rates(torch, ovl, ctx, B, 20)
    res["tuning"]["24x24x24x48"] = ctx.tuning()
    ctx.close()
    res["copy_reference"] = copy_reference(torch)
    return res


def copy_reference(torch, reps=20):
    """What a plain device copy reaches on this GPU (context for the stencil's
    rate): 1 GiB read and 1 GiB written per copy (torch's copy kernel), timed
    with events around reps back-to-back copies."""
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * src.numel() * 4
    del src, dst
    return {"bytes_per_copy": nbytes, "avg_us": 1e3 * ms, "GBps": nbytes / (ms * 1e6),
            "frac_of_peak": nbytes / (ms * 1e6) / HBM_PEAK_GBS}


def cpu_baseline(mscg_iters_per_solve):
    """The oracle (FP64, C stencil + numpy) on a bounded sample of the same
    workload: 96 multi-shift CG iterations (about 15 s on the host) with all
    20 shifts active on the 16^3 x 32 field, scaled by the GPU solve's
    multi-shift iteration count; and the oracle's whole plain-method solve on
    4^4 (c1_solve_seconds), to set beside the GPU's on the same problem."""
    import numpy as np
    import synth
    from oracle import krylov
    from oracle.lattice import WilsonKernel
    from oracle.zolotarev import Zolotarev
    U = synth.gauge_field(DIMS, 2, 0.25)
    k = WilsonKernel(DIMS, U, RHO)
    z = Zolotarev(NZ, 0.6, 8.0 - RHO)
    b = synth.gaussian_source(DIMS, 102)
    iters = 96
    t0 = time.perf_counter()
    krylov.multishift_cg(k.K2s, z.sigma, b, np.full(NZ, 1e-300), maxiter=iters)
    dt = time.perf_counter() - t0
    per_iter = dt / iters
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the whole plain-method solve on 4^4, where the oracle finishes in seconds
    dims1 = (4, 4, 4, 4)
    k1 = WilsonKernel(dims1, synth.gauge_field(dims1, 1, 0.3), RHO)
    w1 = np.linalg.eigvalsh(k1.dense("K"))
    ov1 = krylov.Overlap(krylov.SignFunction(k1, Zolotarev(16, np.abs(w1).min(), np.abs(w1).max())), 0.05)
    t0 = time.perf_counter()
    krylov.gmresr_sumr(ov1, synth.point_source(dims1), TOL, 1e-3)
    c1 = time.perf_counter() - t0
    return {"value": 1.0 / (per_iter * mscg_iters_per_solve), "unit": "solves/s", "cores": threads,
            "c1_solve_seconds": c1,
            "kind": "oracle",
            "sample": f"{iters} multi-shift CG iterations (20 shifts active) of the oracle on the "
                      f"16^3x32 field in {dt:.1f} s, scaled by the {mscg_iters_per_solve} multi-shift "
                      f"iterations of the GPU's FP64 solve (an upper bound on the oracle's rate: fewer "
                      f"shifts stay active in a real solve)"}


C3_DIMS, C3_MU, C3_EPS, C3_SEED = (24, 24, 24, 48), 0.01, 0.25, 3
C3_NAME = "24x24x24x48"
TRAFFIC_C3 = os.path.join(HERE, "profiles", "traffic_overlap_solve_24c48.txt")


def c3_setup(torch, ovl, tuning=None, full_links=False):
    """The 24^3 x 48 workload: links, the Zolotarev interval from Lanczos on
    K^2 (a = 0.95 x its smallest Ritz value, b = 8 - rho, a rigorous bound),
    the coefficients and the twelve spin-colour point sources at the origin."""
    ctx = ovl.Context(C3_DIMS)
    if tuning and C3_NAME in tuning:
        ctx.set_tuning(tuning[C3_NAME])
    if full_links:
        ctx.set_option(ovl.OPT_TWO_ROW_LINKS, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.gauge_generate(C3_SEED, C3_EPS)
    lo, err, hi = ctx.kernel_interval(RHO)
    a, b = 0.95 * lo, 8.0 - RHO
    zolo = ovl.zolotarev_coeffs(NZ, a, b)
    B = [ctx.source(ovl.SRC_POINT, site=0, spin=s, colour=c) for s in range(4) for c in range(3)]
    torch.cuda.synchronize()
    info = {"seconds": time.perf_counter() - t0, "interval": [a, b], "lanczos_lmin": lo, "lanczos_lmin_err": err,
            "lanczos_lmax": hi, "zolotarev_delta": zolo.delta, "n_z": NZ,
            "two_row_links": ctx.gauge_info()[1], "su3_deviation": ctx.gauge_info()[0]}
    return ctx, zolo, B, info


def c3_params(ovl, args, mixed=True, calc=0, defl=1, block=0):
    return ovl.solver_defaults(rho=RHO, mu=C3_MU, tol=TOL, eta_tilde=args.c3_eta, relax_floor=args.relax_cap,
                               f32_threshold=(1e-6 if mixed else 10.0), half_threshold=(3e-3 if mixed else 10.0),
                               max_outer=16, max_middle=6000, max_mscg=20000, use_deflation=defl, eig_calc=calc,
                               n_eig=args.eig_n, m_eig=args.eig_m, eig_eps=args.eig_eps, eig_block=block)


def timed_solve(torch, ctx, b, zolo, p):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st, code = ctx.solve(b, zolo, p)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, st[0].as_dict(), code, x


def true_relres(torch, ctx, b, x, mu, zolo):
    """||b - D x|| / ||b|| with the FP64 operator at sign accuracy 1e-13 (not timed)."""
    Dx, _ = ctx.overlap(x, RHO, mu, zolo, 1e-13)
    return float(torch.linalg.vector_norm(b - Dx) / torch.linalg.vector_norm(b))


def median(xs):
    ys = sorted(xs)
    return ys[len(ys) // 2] if len(ys) % 2 else 0.5 * (ys[len(ys) // 2 - 1] + ys[len(ys) // 2])


def c3_headline(torch, ovl, args, tuning):
    """Set-up, eigSUMR calculating solves, the timed deflated solves, the
    profiled replica and the comparison solves on 24^3 x 48."""
    ctx, zolo, B, setup = c3_setup(torch, ovl, tuning, args.full_links)
    ctx.set_option(ovl.OPT_ADAPTIVE_NZ, 0 if args.fixed_nz else 1)
    ctx.set_option(ovl.OPT_BOUND_PRINTED, 0 if args.bound_text else 1)
    ctx.set_option(ovl.OPT_OUTER_PRINTED, 1 if args.outer_printed else 0)
    n_calc = args.eig_calc
    # eigSUMR calculating solves (Alg. 5 collection at the stricter of the
    # inversion and Sec. 5.1 accuracies, Alg. 6, the three-set step at the end
    # of each) on the first sources, then v^D recomputed in FP64
    ctx.eigspace_set(args.eig_n, args.eig_m, C3_MU)
    calc = []
    if args.eig_block:   # the first n_calc sources in one calculating call, one basis (block eigSUMR)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, sts, code = ctx.solve(torch.stack(B[:n_calc]), zolo, c3_params(ovl, args, True, 1, 1, block=1))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        calc.append({"seconds": dt, "status": code, "sources": n_calc,
                     "sumr_iters_per_source": [st.sumr_iters for st in sts]})
        print(f"[bench] C3 block calculating solve of {n_calc} sources: {dt:.1f} s", file=sys.stderr, flush=True)
    else:
        for i in range(n_calc):
            dt, st, code, _ = timed_solve(torch, ctx, B[i], zolo, c3_params(ovl, args, True, 1, 1))
            calc.append({"seconds": dt, "status": code, **st})
            print(f"[bench] C3 calculating solve {i}: {dt:.1f} s, {st['sumr_iters']} SUMR iterations",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.eigspace_recompute(RHO, zolo, 1e-12)
    torch.cuda.synchronize()
    t_recompute = time.perf_counter() - t0
    info = ctx.eigspace_info()
    ritz = info["ritz"]
    absr = sorted(abs(h) for h in ritz)
    # timed deflated solves: step i solves source (n_calc + i) mod 12
    src = lambda i: B[(n_calc + i) % 12]
    pd = c3_params(ovl, args, True, 0, 1)
    for w in range(args.warmup):
        timed_solve(torch, ctx, src(w), zolo, pd)
    ctx.profile(False)
    steps, x = [], None
    for k in range(args.steps):
        dt, st, code, x = timed_solve(torch, ctx, src(args.warmup + k), zolo, pd)
        steps.append({"seconds": dt, "status": code, **st})
    t_total = sum(s["seconds"] for s in steps)
    last = src(args.warmup + args.steps - 1)
    res_last = true_relres(torch, ctx, last, x, C3_MU, zolo)
    print(f"[bench] C3 deflated mixed: {args.steps} solves in {t_total:.2f} s", file=sys.stderr, flush=True)
    # profiled replica of one timed solve (events on every stencil and shift-update launch)
    ctx.profile(True)
    dtp, stp, _, _ = timed_solve(torch, ctx, src(args.warmup + args.steps), zolo, pd)
    prof = read_prof(ctx, ovl)
    ctx.profile(False)
    # comparisons on the first three timed sources: undeflated mixed, deflated FP64
    cmp_src = [src(args.warmup + k) for k in range(3)]
    defl_t = [s["seconds"] for s in steps[:3]] if len(steps) >= 3 else [s["seconds"] for s in steps]
    defl_it = [s["sumr_iters"] for s in steps[:3]]
    und = [timed_solve(torch, ctx, b, zolo, c3_params(ovl, args, True, 0, 0)) for b in cmp_src]
    print("[bench] C3 undeflated mixed comparison done", file=sys.stderr, flush=True)
    f64 = [] if args.no_fp64 else [timed_solve(torch, ctx, b, zolo, c3_params(ovl, args, False, 0, 1))
                                   for b in cmp_src]
    print("[bench] C3 FP64 comparison done", file=sys.stderr, flush=True)
    res_f64 = true_relres(torch, ctx, cmp_src[-1], f64[-1][3], C3_MU, zolo) if f64 else None
    res_und = true_relres(torch, ctx, cmp_src[-1], und[-1][3], C3_MU, zolo)
    t_und, t_def = median([u[0] for u in und]), median(defl_t)
    it_und, it_def = median([u[1]["sumr_iters"] for u in und]), median(defl_it)
    t_calc = sum(c["seconds"] for c in calc)
    extra = t_calc + t_recompute - n_calc * t_und   # the calculating solves solved n_calc sources too
    gain = t_und - t_def
    out = {
        "setup": setup,
        "eigsumr": {"n_eig": args.eig_n, "m_eig": args.eig_m, "eig_eps": args.eig_eps,
                    "calculating": "one block call" if args.eig_block else "one source after another",
                    "calculating_solves": calc,
                    "calculating_seconds": t_calc, "recompute_fp64_seconds": t_recompute,
                    "diagonalisations": info["ndiag"], "ritz": ritz, "residuals": info["resid"],
                    "bound": "chi scales the bound" if args.bound_text else "as printed (chi on the square root)",
                    "zolotarev_order": "20 in every sign call" if args.fixed_nz else
                    "per sign call: the fewest poles n <= 20 with Delta(n) <= eta / 4 (Sec. 3)",
                    "outer_products": "||D u - c|| < eps ||b|| ||u|| / ||r|| (Alg. 3 as printed)"
                    if args.outer_printed else "||D u - c|| <= eps ||b|| / 4"},
        "steps": steps, "seconds_timed": t_total, "true_relres_last_step": res_last,
        "profiled_replica_seconds": dtp, "profiled_replica_stats": stp,
        "undeflated_mixed": {"median_seconds": t_und, "solves_per_s": 1.0 / t_und, "median_sumr_iters": it_und,
                             "runs": [{"seconds": u[0], "status": u[2], **u[1]} for u in und],
                             "true_relres_last": res_und},
        "deflated_fp64": ({"median_seconds": median([f[0] for f in f64]), "solves_per_s": 1.0 / median([f[0] for f in f64]),
                           "runs": [{"seconds": f[0], "status": f[2], **f[1]} for f in f64],
                           "true_relres_last": res_f64} if f64 else None),
        "deflation": {"sumr_iteration_gain": it_und / it_def if it_def else None,
                      "time_gain": t_und / t_def if t_def else None,
                      # |h| of gamma_5 D(mu) is at least mu; a Ritz value inside
                      # (-mu, mu) is a mixture of a +- pair, so mu bounds the lower end
                      "eigenvalue_ratio": absr[-1] / max(absr[0], C3_MU) if absr else None,
                      "abs_ritz_min_max": [absr[0], absr[-1]] if absr else None,
                      "setup_beyond_plain_solves_s": extra,
                      "break_even_sources": (extra / gain) if gain > 0 else None,
                      "solves_per_s_including_setup_12_sources":
                          12.0 / (setup["seconds"] + t_calc + t_recompute + (12 - n_calc) * t_def)},
        "tuning": ctx.tuning(),
    }
    if args.batch12:
        # the twelve sources deflated in one batched call (right-hand sides
        # grouped by the precision their sign calls need)
        Bs = torch.stack(B)
        dt, _, code, X = timed_solve(torch, ctx, Bs, zolo, pd)
        res = [true_relres(torch, ctx, Bs[f], X[f], C3_MU, zolo) for f in range(12)]
        out["batch12_deflated"] = {"status": code, "seconds": dt, "solves_per_s": 12 / dt,
                                   "single_solves_per_s": 1.0 / t_def, "max_true_relres": max(res)}
        print("[bench] C3 batch of 12 done", file=sys.stderr, flush=True)
    return ctx, zolo, out, prof


def c2_secondary(torch, ovl, args, tuning):
    """The 16^3 x 32 plain method (the paper's inverter without deflation):
    mixed ladder (steps 3, warm-up 1) and all-FP64 (median of three)."""
    ctx, zolo, b = setup_c2(ovl, tuning)
    dt_mix, st_mix, prof_mix, x_mix, _ = time_solves(torch, ctx, ovl, b, zolo,
                                                    solve_params(ovl, True, args.half_threshold), 3, 1)
    f64 = [timed_solve(torch, ctx, b, zolo, solve_params(ovl, False)) for _ in range(3)]
    t64 = median([f[0] for f in f64])
    ks = kernel_summary(prof_mix)
    dom = max(ks, key=lambda k: ks[k]["ms"])
    out = {"workload": "overlap solve 16^3x32, rho=1.4, mu=0.02, N_Z=20, 10 exact kernel modes, Gaussian "
                       "source, GMRESR(relSUMR) to 1e-10 (middle solves to 3e-3)",
           "mixed_solves_per_s": 3 / dt_mix, "fp64_solves_per_s": 1.0 / t64, "mixed_over_fp64": (3 / dt_mix) * t64,
           "true_relres": {"mixed": true_relres(torch, ctx, b, x_mix, MU, zolo),
                           "fp64": true_relres(torch, ctx, b, f64[-1][3], MU, zolo)},
           "solve_stats": {"mixed": st_mix[-1], "fp64": f64[-1][1]},
           "kernels_mixed": ks,
           "dominant_kernel": {"kernel": dom, "achieved_GBps": ks[dom]["GBps"], "avg_us": ks[dom]["avg_us"],
                               "bound": "mall",
                               "note": "16^3x32: fields and links fit in the 256 MB Infinity Cache"},
           "tuning": ctx.tuning()}
    ctx.close()
    return out


def sign_methods_leg(torch, ovl, tuning=None):
    """sign(K) psi in FP64 by the multi-shift CG over the 20 Zolotarev poles
    and by the two-pass Lanczos method, on 16^3 x 32 (ten exact kernel modes)
    and 24^3 x 48 (Lanczos interval), Gaussian source, at sign accuracies
    1e-10 and 1e-4: wall time, steps, and the difference of the two results."""
    out = {}
    for name in ("16x16x16x32", "24x24x24x48"):
        if name == "16x16x16x32":
            ctx, zolo, b = setup_c2(ovl, tuning)
        else:
            ctx, zolo, _, _ = c3_setup(torch, ovl, tuning)
            b = ctx.source(ovl.SRC_GAUSS, seed=102)
        res = {}
        for eta in (1e-10, 1e-4):
            ctx.sign(b, RHO, zolo, eta)   # warm-up (launch tuning)
            ctx.sign_lanczos(b, RHO, zolo, eta)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s1, st1 = ctx.sign(b, RHO, zolo, eta)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s2, st2 = ctx.sign_lanczos(b, RHO, zolo, eta)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            diff = float(torch.linalg.vector_norm(s1 - s2) / torch.linalg.vector_norm(b))
            res[f"{eta:g}"] = {"mscg": {"seconds": t1 - t0, "iterations": st1.mscg_iters,
                                        "us_per_iteration": 1e6 * (t1 - t0) / max(1, st1.mscg_iters)},
                               "lanczos": {"seconds": t2 - t1, "steps_first_pass": st2.mscg_iters,
                                           "us_per_step_both_passes": 1e6 * (t2 - t1) / max(1, st2.mscg_iters)},
                               "relative_difference": diff}
        out[name] = res
        ctx.close()
    return out


def variant_sweep(torch, ovl, reps=10):
    """Every admissible stencil launch variant forced through the tuning table:
    the hopping stencil over twelve fields of 24^3 x 48 (links seed 3, links
    read once per launch in the algorithmic bytes) and over one field of
    32^3 x 64 (links seed 5), FP32 and FP16 storage, one warm-up launch and
    `reps` timed launches each (HIP events on the dispatches).  Under
    rocprofv3 --pmc the dispatches come in the order listed here, `reps + 1`
    per variant."""
    out = []
    for name, dims, seed, nf in (("24^3x48, 12 fields", (24, 24, 24, 48), 3, 12),
                                 ("32^3x64, 1 field", (32, 32, 32, 64), 5, 1)):
        ctx = ovl.Context(dims)
        ctx.gauge_generate(seed, 0.25)
        if nf == 1:
            psi = ctx.source(ovl.SRC_GAUSS, seed=7)
        else:
            psi = torch.stack([ctx.source(ovl.SRC_GAUSS, seed=300 + f) for f in range(nf)])
        for prec in (ovl.F32, ovl.HALF):
            for v in range(ovl.N_STENCIL_VARIANTS):
                try:
                    ctx.set_tuning({(prec * 8 + 0) * 64 + nf: v})   # the hopping epilogue, nf fields
                except ovl.OvlError:
                    continue   # not admissible on this lattice or in this precision
                ctx.wilson_dslash(psi, prec)
                torch.cuda.synchronize()
                ctx.profile(True)
                for _ in range(reps):
                    ctx.wilson_dslash(psi, prec)
                torch.cuda.synchronize()
                p = ctx.profile_read(ovl.KERN_STENCIL, prec)
                ctx.profile(False)
                out.append({"lattice": name, "prec": PREC_NAMES[prec], "variant": v, "launches": p["launches"],
                            "avg_us": 1e3 * p["ms"] / p["launches"], "bytes_per_launch": p["bytes"] / p["launches"],
                            "GBps": p["bytes"] / (p["ms"] * 1e6)})
                print(f"[bench] variant sweep {name} {PREC_NAMES[prec]} variant {v}: "
                      f"{out[-1]['avg_us']:.1f} us, {out[-1]['GBps']:.0f} GB/s", file=sys.stderr, flush=True)
        ctx.close()
    return out


def stream_ceiling(torch, ovl):
    """The library's own streaming kernels on 1 GiB buffers: copy (1 GiB
    read + 1 GiB written per launch) and read-only."""
    ctx = ovl.Context((4, 4, 4, 4))
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    ms_c = ctx.stream_bench(0, src, dst, 20)
    ms_r = ctx.stream_bench(1, src, dst, 20)
    nb = src.numel() * 8
    del src, dst
    ctx.close()
    return {"copy": {"bytes_per_launch": 2 * nb, "avg_us": 1e3 * ms_c, "GBps": 2 * nb / (ms_c * 1e6),
                     "frac_of_peak": 2 * nb / (ms_c * 1e6) / HBM_PEAK_GBS},
            "read": {"bytes_per_launch": nb, "avg_us": 1e3 * ms_r, "GBps": nb / (ms_r * 1e6),
                     "frac_of_peak": nb / (ms_r * 1e6) / HBM_PEAK_GBS}}


def cpu_baseline_c3(mscg_iters_per_solve, samples=3, iters=6):
    """The oracle (FP64, C stencil and vector updates, numpy) on a bounded
    sample of the headline workload: `iters` multi-shift CG iterations with
    all 20 shifts active on the 24^3 x 48 field, three times (the median),
    scaled by the multi-shift iteration count of the GPU's FP64 deflated solve
    of the same workload (an upper bound on the oracle's rate: fewer shifts
    stay active in a real solve)."""
    import numpy as np
    import synth
    from oracle import krylov
    from oracle.lattice import WilsonKernel
    from oracle.zolotarev import Zolotarev
    U = synth.gauge_field(C3_DIMS, C3_SEED, C3_EPS)
    k = WilsonKernel(C3_DIMS, U, RHO)
    z = Zolotarev(NZ, 0.588, 8.0 - RHO)
    b = synth.point_source(C3_DIMS)
    per = []
    for _ in range(samples):
        t0 = time.perf_counter()
        krylov.multishift_cg(k.K2s, z.sigma, b, np.full(NZ, 1e-300), maxiter=iters)
        per.append((time.perf_counter() - t0) / iters)
    per_iter = median(per)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / (per_iter * mscg_iters_per_solve), "unit": "solves/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{iters} multi-shift CG iterations (20 shifts active) of the oracle on the 24^3x48 "
                      f"field, median of {samples} runs: {per_iter:.3f} s per iteration, scaled by the "
                      f"{mscg_iters_per_solve} multi-shift iterations of the GPU's FP64 deflated solve "
                      f"(an upper bound on the oracle's rate: fewer shifts stay active in a real solve)"}


def main():
    args = parse()
    if not 1 <= args.eig_calc <= 11:
        print("bench.py: --eig-calc takes 1 .. 11 (the twelve spin-colour sources, at least one left to time)",
              file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU (no multi-GPU path); --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1501_01855_amd as ovl

    tuning = json.loads(args.tuning) if args.tuning else None
    if args.profile_run:
        profile_run(torch, ovl, tuning, args)
        return
    if args.variant_sweep:
        print(json.dumps({"variant_sweep": variant_sweep(torch, ovl)}), flush=True)
        return
    ctx, zolo, c3, prof = c3_headline(torch, ovl, args, tuning)
    ks = kernel_summary(prof)
    dom = max(ks, key=lambda k: ks[k]["ms"])
    d = ks[dom]
    traffic, traffic_note = read_traffic(dom, TRAFFIC_C3)
    valu, valu_note = read_counter("valu", dom, TRAFFIC_C3)
    issue = None
    if valu is not None:   # vector instruction issue: one wave instruction per clock per CU
        rate = valu / (d["avg_us"] * 1e-6) / 1e9
        issue = {"valu_wave_instructions_per_launch": valu, "achieved": rate, "peak": VALU_ISSUE_PEAK,
                 "unit": "G wave-instructions/s", "frac": rate / VALU_ISSUE_PEAK, "source": valu_note}
    roofline = {"bound": "hbm", "kernel": dom, "achieved": d["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["GBps"] / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": d["bytes_per_launch"], "avg_us": d["avg_us"],
                "traffic_note": traffic_note, "issue": issue,
                "working_set": "24^3x48: the multi-shift CG's fields (25 x 34.5 MB in FP16 storage) and links "
                               "exceed the 256 MB Infinity Cache"}
    t_total = c3.pop("seconds_timed")
    f64 = c3.get("deflated_fp64")
    value = args.steps / t_total
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32/f64",
        "data": "synthetic",
        "config": {"workload": "overlap solve 24^3x48 (links exp(i 0.25 A), seed 3), rho=1.4, mu=0.01, Zolotarev "
                               "sign function (" + ("20 poles" if args.fixed_nz else "at most 20 poles, order per call "
                               "from its accuracy") + ") on the Lanczos interval of |K|, eigSUMR deflation with "
                               f"{args.eig_n} eigenvectors (m={args.eig_m}, {args.eig_calc} calculating solves"
                               + (" in one block call" if args.eig_block else "") + "), one "
                               "spin-colour point source per step (cycling over the 12), mixed precision, "
                               f"GMRESR(relSUMR) to 1e-10 (middle solves to {args.c3_eta:g})",
                   "global_batch": 1, "lattice": C3_NAME, "parallelism": "single GPU"},
        "fp64_solves_per_s": f64["solves_per_s"] if f64 else None,
        "mixed_over_fp64": (value / f64["solves_per_s"]) if f64 else None,
        "kernels_mixed": ks,
        "kernel_timing": "HIP events on each launch's dispatch packet, in one profiled replica of a timed "
                         "solve (same kernels and launch shapes)",
        "roofline": roofline,
        "c3": c3,
    }
    out["tuning"] = {C3_NAME: c3.pop("tuning")}
    ctx.close()
    if not args.headline_only:   # the secondary workloads; optional legs below run either way
        out["c2_16c32"] = c2_secondary(torch, ovl, args, tuning)
        out["tuning"]["16x16x16x32"] = out["c2_16c32"].pop("tuning")
        print("[bench] 16^3x32 plain method done", file=sys.stderr, flush=True)
        out["dslash_hbm"] = dslash_alone(torch, ovl, tuning)
        for name, t in out["dslash_hbm"].pop("tuning").items():   # merged: 24^3x48 holds the solve's choices too
            out["tuning"].setdefault(name, {}).update(t)
        out["dslash_hbm"]["stream_ceiling"] = stream_ceiling(torch, ovl)
        print("[bench] stand-alone stencil and streaming ceiling done", file=sys.stderr, flush=True)
    if args.extras:
        out["uneven_instances"] = uneven_leg(torch, ovl)
        print("[bench] uneven instances done", file=sys.stderr, flush=True)
        out["c1_plain_4c4"] = c1_leg(torch, ovl)
        out["adjoint"] = adjoint_leg(torch, ovl)
        print("[bench] 4^4 and adjoint legs done", file=sys.stderr, flush=True)
    if args.sign_methods or args.extras:
        out["sign_methods"] = sign_methods_leg(torch, ovl, tuning)
        print("[bench] sign-function methods done", file=sys.stderr, flush=True)
    if args.eigcg:
        out["eigcg_16c32"] = eigcg_leg(torch, ovl, args.eigcg_calc)
    if args.eigsolve:
        out["eigsolve_16c32"] = eigsolve_leg(torch, ovl)
    if not args.no_cpu and not args.headline_only:
        it = f64["runs"][len(f64["runs"]) // 2]["mscg_iters"] if f64 else c3["undeflated_mixed"]["runs"][0]["mscg_iters"]
        out["cpu_baseline"] = cpu_baseline_c3(it)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
